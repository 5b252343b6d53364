"""closure_noalloc, the closure entry point that allocates nothing (its
working memory is the library's static per-device scratch), against
closure() on the same inputs: two calls in a row per kind, the second on a
smaller matrix (so the scratch holds the first call's leftovers), every entry
compared; the first pair also against the oracle.  Sizes whose working memory
exceeds the scratch are refused before anything is enqueued."""
import ctypes

import numpy as np
import pytest

import oracle
import paper_1705_08743_amd as sr
import synthgen
from gpu_util import S_OF, rand_antidist, rand_bits, rand_dist, set_oracle_threads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    set_oracle_threads()


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _abi_noalloc(kind, T, D, flags=0):
    """closure_noalloc called through the C ABI (ctypes), not the binding."""
    ld = T.stride(0)
    return sr.lib().closure_noalloc(kind, T.data_ptr(), ld, D, flags, _stream())


def _input(kind, D, seed):
    gen = synthgen.generator(seed)
    if kind == sr.SR_BOOL:
        bits = rand_bits(D, D, gen, p=2.0 / max(D, 1))
        return synthgen.pack_bits(bits, synthgen.aligned_ld_words(D))
    if kind in (sr.SR_DISTANCE_U8, sr.SR_DISTANCE_U16, sr.SR_DISTANCE_U32):
        return rand_dist(D, D, kind, gen, p=0.05, wmax=S_OF[kind] // 8)
    return rand_antidist(D, D, kind, gen, p=0.05, wmax=S_OF[kind] // 8)


def _both(kind, A, D, flags=0):
    """(closure_noalloc result, closure result) on copies of A."""
    cols = D if kind == sr.SR_BOOL else None
    T1 = sr.to_device(kind, A, cols=cols)
    T2 = sr.clone(T1)
    assert _abi_noalloc(kind, T1, D, flags) == sr.SR_OK, sr.lib().sr_last_error().decode()
    sr.closure(kind, T2, D=D, flags=flags)
    torch.cuda.synchronize()
    return sr.to_host(T1), sr.to_host(T2)


def _oracle(kind, A, D):
    if kind == sr.SR_BOOL:
        return oracle.bool_closure_words(A, D)
    if kind in (sr.SR_DISTANCE_U8, sr.SR_DISTANCE_U16, sr.SR_DISTANCE_U32):
        return oracle.dist_closure(A, S_OF[kind])
    return oracle.ad_closure(A, S_OF[kind])


def _same(kind, got, want, D):
    if kind == sr.SR_BOOL:
        nw = (D + 63) // 64
        return np.array_equal(got[:, :nw], want[:, :nw])
    return np.array_equal(got[:, :D].astype(np.int64), want[:, :D].astype(np.int64))


# (kind, first D, second D): the first sizes take the working memory of the
# squaring closure (uint16 1024, uint32 700), of big pivot blocks (uint16
# distances 1500), of the uint8 working copy plus big blocks (2100) or the
# whole 32 MiB (uint8 4096, the loop), or the transposed pivot rows of the
# matrix-core update (Boolean 2100; first, so that in a fresh process it
# runs before any call has made the second stream: every phase on the
# caller's stream); Boolean 1100 needs none.
CASES = [
    (sr.SR_BOOL, 2100, 1100),
    (sr.SR_ANTIDIST_U16, 1024, 700),
    (sr.SR_ANTIDIST_U8, 2100, 300),
    (sr.SR_ANTIDIST_U8, 4096, 1000),
    (sr.SR_ANTIDIST_U32, 700, 300),
    (sr.SR_DISTANCE_U16, 1500, 250),
    (sr.SR_DISTANCE_U8, 900, 129),
    (sr.SR_BOOL, 1100, 100),
]


@pytest.mark.parametrize("kind,D1,D2", CASES)
def test_noalloc_equals_closure(kind, D1, D2):
    A1 = _input(kind, D1, 9000 + D1)
    got1, ref1 = _both(kind, A1, D1)
    assert _same(kind, got1, ref1, D1), "first call differs from closure()"
    if D1 <= 2100:
        assert _same(kind, got1, _oracle(kind, A1, D1), D1), "first call differs from the oracle"
    A2 = _input(kind, D2, 9100 + D2)
    got2, ref2 = _both(kind, A2, D2)
    assert _same(kind, got2, ref2, D2), "second (smaller) call differs from closure()"
    assert _same(kind, got2, _oracle(kind, A2, D2), D2)


@pytest.mark.parametrize("flags", [sr.SR_REFLEXIVE, sr.SR_CLOSURE_SQUARING,
                                   sr.SR_CLOSURE_WARSHALL, sr.SR_CLOSURE_BIG_BLOCKS])
def test_noalloc_forced_methods(flags):
    kind = sr.SR_ANTIDIST_U16
    for D in (1300, 260):
        A = _input(kind, D, 9200 + D + flags)
        got, ref = _both(kind, A, D, flags)
        assert _same(kind, got, ref, D)


def test_noalloc_refuses_oversized_work():
    """A uint8 matrix above 4096 vertices needs more than the 32 MiB scratch:
    SR_EINVAL before anything is enqueued (the matrix is left as it was)."""
    kind = sr.SR_ANTIDIST_U8
    D = 4100
    A = _input(kind, D, 9300)
    T = sr.to_device(kind, A)
    assert _abi_noalloc(kind, T, D) == sr.SR_EINVAL
    assert "static scratch" in sr.lib().sr_last_error().decode()
    torch.cuda.synchronize()
    assert np.array_equal(sr.to_host(T)[:, :D], A[:, :D])
