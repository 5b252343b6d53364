"""Autotuning: sr_autotune_closure / sr_autotune_mul time the exact methods
that apply, keep the fastest per size class, and the default calls then use
it; every method gives the oracle's result, so the tests check that the
choice is a valid method and that closure() / semiring_mul() after tuning
still equal the oracle."""
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
    yield
    sr.autotune_clear()
    torch.cuda.synchronize()


CLOSURE_METHODS = {sr.SR_CLOSURE_WARSHALL, sr.SR_CLOSURE_SQUARING, sr.SR_CLOSURE_BIG_BLOCKS,
                   sr.SR_CLOSURE_WARSHALL | sr.SR_BOOL_BITWISE,
                   sr.SR_CLOSURE_WARSHALL | sr.SR_BOOL_M4R,
                   sr.SR_CLOSURE_WARSHALL | sr.SR_BOOL_MFMA}


@pytest.mark.parametrize("kind,D", [(sr.SR_ANTIDIST_U16, 700), (sr.SR_ANTIDIST_U8, 1500),
                                    (sr.SR_ANTIDIST_U32, 300), (sr.SR_DISTANCE_U16, 2100),
                                    (sr.SR_BOOL, 1100)])
def test_autotune_closure_then_default_equals_oracle(kind, D):
    chosen = sr.autotune_closure(kind, D)
    assert chosen in CLOSURE_METHODS
    if kind != sr.SR_BOOL:
        assert not chosen & (sr.SR_BOOL_BITWISE | sr.SR_BOOL_M4R | sr.SR_BOOL_MFMA)
    gen = synthgen.generator(9970 + kind + D)
    if kind == sr.SR_BOOL:
        A = rand_bits(D, D, gen, 2.0 / D)
        T = sr.to_device(kind, synthgen.pack_bits(A, synthgen.aligned_ld_words(D)), cols=D)
        want = oracle.bool_closure(A)
    elif kind == sr.SR_DISTANCE_U16:
        A = rand_dist(D, D, kind, gen, p=2.0 / D, wmax=S_OF[kind] // 6)
        T = sr.to_device(kind, A)
        want = oracle.dist_closure(A, S_OF[kind])
    else:
        A = rand_antidist(D, D, kind, gen, p=2.0 / D, wmax=S_OF[kind] // 6)
        T = sr.to_device(kind, A)
        want = oracle.ad_closure(A, S_OF[kind])
    T2 = sr.clone(T)
    sr.closure(kind, T, D=D)              # the tuned default
    sr.closure(kind, T2, D=D, flags=chosen)  # the same method, named
    torch.cuda.synchronize()
    for t in (T, T2):
        h = sr.to_host(t)
        got = synthgen.unpack_bits(h, D) if kind == sr.SR_BOOL else h.astype(np.int64)
        assert np.array_equal(got, want)


def test_autotune_bool_mul_then_default_equals_oracle():
    R, K, N = 1000, 2000, 3000
    chosen = sr.autotune_mul(sr.SR_BOOL, R, K, N)
    assert chosen in (sr.SR_BOOL_BITWISE, sr.SR_BOOL_M4R, sr.SR_BOOL_MFMA)
    gen = synthgen.generator(9980)
    A = synthgen.pack_bits(rand_bits(R, K, gen, 0.002), synthgen.aligned_ld_words(K))
    B = synthgen.pack_bits(rand_bits(K, N, gen, 0.002), synthgen.aligned_ld_words(N))
    dA = sr.to_device(sr.SR_BOOL, A, cols=K)
    dB = sr.to_device(sr.SR_BOOL, B, cols=N)
    C = sr.empty(sr.SR_BOOL, R, N)
    sr.semiring_mul(sr.SR_BOOL, C, dA, dB, K=K, N=N)
    torch.cuda.synchronize()
    nw = (N + 63) // 64
    want = oracle.bool_mul_words(A, B, K, N)
    assert np.array_equal(sr.to_host(C)[:, :nw], want[:, :nw])
    with pytest.raises(sr.SemiringError) as e:
        sr.autotune_mul(sr.SR_ANTIDIST_U16, 8, 8, 8)
    assert e.value.code == sr.SR_EUNSUPPORTED


def test_autotune_table_persists(tmp_path):
    """A tuned closure choice (method and, for big blocks, the pivot block)
    survives a save, a clear and a load: the working-memory query and the
    default closure follow it again, and the closure equals the oracle."""
    kind, D = sr.SR_ANTIDIST_U16, 1500
    sr.autotune_clear()
    chosen = sr.autotune_closure(kind, D)
    tuned_bytes = sr.closure_work_bytes(kind, D)
    f = tmp_path / "tune.json"
    sr.autotune_save(str(f))
    sr.autotune_clear()
    sr.autotune_load(str(f))
    assert sr.closure_work_bytes(kind, D) == tuned_bytes
    assert '"arch": "gfx950"' in f.read_text()
    gen = synthgen.generator(9990)
    A = rand_antidist(D, D, kind, gen, p=2.0 / D, wmax=S_OF[kind] // 6)
    T = sr.to_device(kind, A)
    sr.closure(kind, T)
    torch.cuda.synchronize()
    assert np.array_equal(sr.to_host(T).astype(np.int64), oracle.ad_closure(A, S_OF[kind])), chosen
    sr.autotune_clear()

