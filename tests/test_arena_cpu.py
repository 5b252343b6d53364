"""Layout of BatchArena (host logic; a CPU buffer stands in for device
memory): every matrix 256-byte aligned, row strides padded to 128 bytes,
matrices disjoint, views and the host image agree."""
import numpy as np
import pytest

import paper_1705_08743_amd as sr

torch = pytest.importorskip("torch")


@pytest.mark.parametrize("kind", [sr.SR_ANTIDIST_U8, sr.SR_ANTIDIST_U16])
def test_arena_layout(kind):
    sizes = [0, 1, 63, 64, 65, 130, 7, 0, 300]
    a = sr.BatchArena(kind, sizes, device="cpu")
    es = 1 if kind == sr.SR_ANTIDIST_U8 else 2
    base = a.buf.data_ptr()
    spans = []
    for i, n in enumerate(sizes):
        assert a._ptrs[i] == base + a.offsets[i]
        assert a.offsets[i] % 256 == 0
        assert (a.lds[i] * es) % 128 == 0 and a.lds[i] >= n
        assert a._dims[i] == n
        spans.append((a.offsets[i], a.offsets[i] + n * a.lds[i] * es))
        v = a.view(i)
        assert tuple(v.shape) == (n, n)
        if n > 1:
            assert v.stride(0) == a.lds[i]
            assert v.data_ptr() == a._ptrs[i]
    spans.sort()
    for (lo0, hi0), (lo1, hi1) in zip(spans, spans[1:]):
        assert hi0 <= lo1
    assert spans[-1][1] <= a.buf.numel()


def test_arena_image_roundtrip():
    kind = sr.SR_ANTIDIST_U16
    gen = np.random.default_rng(3)
    sizes = [5, 0, 70, 33]
    mats = [gen.integers(0, 65536, size=(n, n), dtype=np.uint16) for n in sizes]
    a = sr.BatchArena(kind, sizes, device="cpu")
    a.load(mats)
    for i, m in enumerate(mats):
        assert np.array_equal(a.view(i).numpy(), m)
    b = sr.BatchArena(kind, sizes, device="cpu")
    b.copy_(a)
    assert torch.equal(a.buf, b.buf)
    with pytest.raises(ValueError):
        b.copy_(sr.BatchArena(kind, [5, 0, 70, 34], device="cpu"))
    with pytest.raises(ValueError):
        a.load([mats[0], mats[2], mats[1], mats[3]])


def test_arena_boolean_layout_and_image():
    """Boolean arenas: rows of ceil(n / 64) words padded to an even count,
    256-byte aligned matrices, word views and the host image agree."""
    sizes = [0, 1, 63, 64, 65, 129, 200]
    gen = np.random.default_rng(5)
    a = sr.BatchArena(sr.SR_BOOL, sizes, device="cpu")
    spans = []
    for i, n in enumerate(sizes):
        w = -(-n // 64)
        assert a.offsets[i] % 256 == 0
        assert a.lds[i] % 2 == 0 and a.lds[i] >= max(w, 2)
        assert tuple(a.view(i).shape) == (n, w)
        spans.append((a.offsets[i], a.offsets[i] + n * a.lds[i] * 8))
    spans.sort()
    for (lo0, hi0), (lo1, hi1) in zip(spans, spans[1:]):
        assert hi0 <= lo1
    mats = [gen.integers(0, 2 ** 63, size=(n, -(-n // 64)), dtype=np.uint64) for n in sizes]
    a.load(mats)
    for i, m in enumerate(mats):
        assert np.array_equal(a.view(i).numpy().view(np.uint64), m)
