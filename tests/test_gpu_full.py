"""Parity at the benchmark's full sizes, in the launch configuration bench.py
times (default flags: phases overlapped on two streams).

Every entry of every result is compared with the oracle's own loops (the
Warshall loop of Sec. II / Sec. III, the multiplication algorithm, the
bit-packed Boolean loops), run once on all host threads the process may use.
Each entry of a closure is fixed by eq. (trcl) and each product entry by the
product's definition, so the comparison is exact equality.  Invariants on
the GPU result (T >= A, overlapped schedule = serial schedule) are extras.
"""
import numpy as np
import pytest

import oracle
import paper_1705_08743_amd as sr
import synthgen
from gpu_util import set_oracle_threads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    set_oracle_threads()


def _close(kind, A, flags=0):
    T = sr.to_device(kind, A)
    sr.closure(kind, T, flags=flags)
    torch.cuda.synchronize()
    return sr.to_host(T)


def _headline_input(kind, D):
    if kind == sr.SR_ANTIDIST_U16:
        return synthgen.cfg_antidist(D=D)[:, :D], 65535
    return synthgen.cfg_antidist_u8(D=D)[:, :D], 255


@pytest.mark.parametrize("kind", [sr.SR_ANTIDIST_U16, sr.SR_ANTIDIST_U8])
def test_headline_closure_d8192(kind):
    """D = 8192 closure (uint16 headline and its uint8 variant): every entry
    against the oracle's Warshall loop, both schedules."""
    D = 8192
    A, S = _headline_input(kind, D)
    got = _close(kind, A)
    want = oracle.ad_closure(A, S)
    assert np.array_equal(got.astype(np.int32), want)
    got_serial = _close(kind, A, sr.SR_SERIAL_PHASES)
    assert np.array_equal(got_serial.astype(np.int32), want)
    assert (got >= A).all()


@pytest.mark.parametrize("kind,D", [(sr.SR_ANTIDIST_U16, 7001), (sr.SR_ANTIDIST_U8, 6500)])
def test_closure_ragged_above_6144(kind, D):
    """Above 6144 vertices the lookahead runs as whole-K launches; a ragged
    last pivot block (7001 = 54 * 128 + 89; 6500 = 50 * 128 + 100) leaves a
    partial last column chunk.  Every entry against the oracle."""
    A, S = _headline_input(kind, D)
    want = oracle.ad_closure(A, S)
    assert np.array_equal(_close(kind, A).astype(np.int32), want)


def test_distance_closure_d8192():
    """The headline input as a distance matrix (entries = distances, S = no
    path), closed with min and saturating +: every entry against the
    oracle's distance Warshall loop; the reflexive form has a zero diagonal
    and the same off-diagonal entries."""
    D = 8192
    S = 65535
    kind = sr.SR_DISTANCE_U16
    A = (S - synthgen.cfg_antidist(D=D)[:, :D].astype(np.int64)).astype(np.uint16)
    T = sr.to_device(kind, A)
    T2 = sr.clone(T)
    sr.closure(kind, T)
    sr.closure(kind, T2, flags=sr.SR_REFLEXIVE)
    torch.cuda.synchronize()
    got = sr.to_host(T)
    want = oracle.dist_closure(A, S)
    assert np.array_equal(got.astype(np.int32), want)
    del want
    got2 = sr.to_host(T2)
    assert (np.diagonal(got2) == 0).all()
    off = ~np.eye(D, dtype=bool)
    assert np.array_equal(got2[off], got[off])


def test_u32_closure_d8192():
    """The headline distances with 32-bit entries (S = 2^32 - 1): every
    entry against the oracle's int64 Warshall loop."""
    D = 8192
    S = 2 ** 32 - 1
    A16 = synthgen.cfg_antidist(D=D)[:, :D].astype(np.int64)
    A = np.where(A16 > 0, S - (65535 - A16), 0).astype(np.uint32)
    del A16
    got = _close(sr.SR_ANTIDIST_U32, A)
    want = oracle.ad_closure(A, S)
    assert np.array_equal(got.astype(np.int64), want)


def test_product_d8192():
    """uint16 product A * B of two D = 8192 graphs: every entry against the
    oracle's multiplication loop."""
    D = 8192
    A = synthgen.cfg_antidist(D=D, which=0)[:, :D]
    B = synthgen.cfg_antidist(D=D, which=1)[:, :D]
    C = sr.empty(sr.SR_ANTIDIST_U16, D, D)
    sr.semiring_mul(sr.SR_ANTIDIST_U16, C, sr.to_device(sr.SR_ANTIDIST_U16, A),
                    sr.to_device(sr.SR_ANTIDIST_U16, B))
    torch.cuda.synchronize()
    want = oracle.ad_mul(A, B, 65535)
    assert np.array_equal(sr.to_host(C).astype(np.int32), want)


def test_add_d8192():
    """semiring_add of the two D = 8192 uint16 inputs the HBM benchmark
    times (its streaming form), out of place and in place: every entry
    against the oracle's entrywise maximum."""
    D = 8192
    kind = sr.SR_ANTIDIST_U16
    A = synthgen.cfg_antidist(D=D, which=0)
    B = synthgen.cfg_antidist(D=D, which=1)
    want = oracle.ewise("or", A, B)
    dA, dB = sr.to_device(kind, A), sr.to_device(kind, B)
    C = sr.empty(kind, D, D)
    sr.semiring_add(kind, C, dA, dB)
    torch.cuda.synchronize()
    assert np.array_equal(sr.to_host(C).astype(np.int64), want)
    sr.semiring_add(kind, dB, dA, dB)
    torch.cuda.synchronize()
    assert np.array_equal(sr.to_host(dB).astype(np.int64), want)


@pytest.fixture(scope="module")
def cfg3():
    """The D = 16384 Boolean input and its closure by the oracle's bit-packed
    Warshall loop (computed once for the tests below)."""
    D = 16384
    W = synthgen.cfg_bool16384(D=D)
    return D, W, oracle.bool_closure_words(W, D)


@pytest.mark.parametrize("flags,fmt", [(0, None), (sr.SR_BOOL_BITWISE, None),
                                       (sr.SR_BOOL_M4R, None), (sr.SR_BOOL_MFMA, "f4"),
                                       (sr.SR_BOOL_MFMA, "i8")])
def test_bool_closure_config3(cfg3, flags, fmt, monkeypatch):
    """Boolean D = 16384, mean out-degree 3 plus planted
    strongly connected blocks; every word against the oracle for the default
    bulk update and each forced one (bit-sliced, four-Russians tables, the
    matrix cores with 4-bit float and with int8 operands); padding bits stay
    clear."""
    if fmt:
        monkeypatch.setenv("SR_MFMA_FORMAT", fmt)
    D, W, want = cfg3
    T = sr.to_device(sr.SR_BOOL, W, cols=D)
    sr.closure(sr.SR_BOOL, T, D=D, flags=flags)
    torch.cuda.synchronize()
    got = sr.to_host(T)
    nw = D // 64
    assert np.array_equal(got[:, :nw], want[:, :nw])
    assert synthgen.padding_bits_clear(got, D)


@pytest.mark.parametrize("flags,fmt", [(0, None), (sr.SR_BOOL_BITWISE, None),
                                       (sr.SR_BOOL_MFMA, "f4"), (sr.SR_BOOL_MFMA, "i8")])
def test_bool_product_config3(cfg3, flags, fmt, monkeypatch):
    """The D = 16384 Boolean product A * A on each path: every word
    against the oracle's bit-packed multiplication loop."""
    if fmt:
        monkeypatch.setenv("SR_MFMA_FORMAT", fmt)
    D, W, _ = cfg3
    A = sr.to_device(sr.SR_BOOL, W, cols=D)
    C = sr.empty(sr.SR_BOOL, D, D)
    sr.semiring_mul(sr.SR_BOOL, C, A, A, K=D, N=D, flags=flags)
    torch.cuda.synchronize()
    want = oracle.bool_mul_words(W, W, D, D)
    nw = D // 64
    assert np.array_equal(sr.to_host(C)[:, :nw], want[:, :nw])


def test_bool_product_d8192():
    """Boolean product at D = 8192 (the size picks the four-Russians path):
    every word against the oracle."""
    D = 8192
    gen = synthgen.generator(8192)
    ld = synthgen.aligned_ld_words(D)
    Aw = synthgen.pack_bits((gen.random((D, D)) < 0.002).astype(np.uint8), ld)
    Bw = synthgen.pack_bits((gen.random((D, D)) < 0.002).astype(np.uint8), ld)
    dA, dB = sr.to_device(sr.SR_BOOL, Aw, cols=D), sr.to_device(sr.SR_BOOL, Bw, cols=D)
    C = sr.empty(sr.SR_BOOL, D, D)
    sr.semiring_mul(sr.SR_BOOL, C, dA, dB, K=D, N=D)
    torch.cuda.synchronize()
    want = oracle.bool_mul_words(Aw, Bw, D, D)
    assert np.array_equal(sr.to_host(C)[:, :D // 64], want[:, :D // 64])


@pytest.mark.parametrize("dtype", [np.uint16, np.uint8])
def test_batched_config4_all_graphs(dtype):
    """4096 graphs of log-uniform sizes in [32, 1024],
    closed by one call; every entry of every graph against the oracle."""
    kind = sr.SR_ANTIDIST_U16 if dtype == np.uint16 else sr.SR_ANTIDIST_U8
    S = 65535 if dtype == np.uint16 else 255
    batch = synthgen.cfg_batch()
    mats = [synthgen.encode_antidist(n, r, c, w, dtype) for n, r, c, w in batch]
    arena = sr.BatchArena(kind, [m.shape[0] for m in mats])
    arena.load(mats)
    sr.closure_batched(kind, arena)
    torch.cuda.synchronize()
    img = arena.buf.cpu().numpy()
    es = np.dtype(dtype).itemsize
    bad = []
    for i, m in enumerate(mats):
        n, ld, off = int(arena.sizes[i]), int(arena.lds[i]), int(arena.offsets[i])
        got = img[off:off + n * ld * es].view(dtype).reshape(n, ld)[:, :n]
        if not np.array_equal(got.astype(np.int32), oracle.ad_closure(m, S)):
            bad.append((i, n))
    assert not bad, bad[:10]
