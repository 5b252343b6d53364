"""Bit-exact parity of the HIP library (through the C ABI) with the oracle.

Sizes span several wave tiles, pivot blocks and ragged tails; every
comparison is element by element with tolerance 0 (all arithmetic is integer).
"""
import numpy as np
import pytest

import oracle
import paper_1705_08743_amd as sr
import synthgen
from gpu_util import S_OF, np_dtype, rand_antidist, rand_bits, rand_dist, set_oracle_threads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

AD_KINDS = [sr.SR_ANTIDIST_U16, sr.SR_ANTIDIST_U8]
MUL_SHAPES = [(1, 1, 1), (3, 5, 2), (64, 64, 64), (65, 130, 129), (200, 37, 300),
              (257, 8, 513), (130, 300, 70), (511, 129, 1000)]


@pytest.fixture(scope="module", autouse=True)
def _setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    set_oracle_threads()
    yield
    torch.cuda.synchronize()


def dev(kind, host, cols=None, ld=None):
    """Device copy; ld=None pads rows to 128 bytes, else uses exactly ld."""
    if ld is None:
        return sr.to_device(kind, host, cols)
    dt = {sr.SR_ANTIDIST_U8: torch.uint8, sr.SR_ANTIDIST_U16: torch.uint16,
          sr.SR_BOOL: torch.int64}[kind]
    buf = torch.zeros((max(host.shape[0], 1), ld), dtype=dt, device="cuda")
    w = host.shape[1]
    src = host.view(np.int64) if kind == sr.SR_BOOL else host
    buf[:host.shape[0], :w].copy_(torch.from_numpy(np.ascontiguousarray(src)))
    return buf[:host.shape[0], :w]


def host(t):
    torch.cuda.synchronize()
    return sr.to_host(t)


# ---------------------------------------------------------------------------
# anti-distance product
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kind", AD_KINDS)
@pytest.mark.parametrize("R,K,N", MUL_SHAPES)
def test_ad_mul(kind, R, K, N):
    gen = synthgen.generator(1000 + R * 7 + K * 3 + N)
    A = rand_antidist(R, K, kind, gen, p=0.4)
    B = rand_antidist(K, N, kind, gen, p=0.4)
    C = sr.empty(kind, R, N)
    sr.semiring_mul(kind, C, dev(kind, A), dev(kind, B))
    want = oracle.ad_mul(A, B, S_OF[kind])
    assert np.array_equal(host(C).astype(np.int64), want)


@pytest.mark.parametrize("kind", AD_KINDS)
def test_ad_mul_accumulate_and_k0(kind):
    gen = synthgen.generator(1001)
    A = rand_antidist(70, 45, kind, gen)
    B = rand_antidist(45, 90, kind, gen)
    C0 = rand_antidist(70, 90, kind, gen, p=0.5)
    C = dev(kind, C0)
    sr.semiring_mul(kind, C, dev(kind, A), dev(kind, B), flags=sr.SR_ACCUMULATE)
    want = oracle.ad_mul(A, B, S_OF[kind], C=C0)
    assert np.array_equal(host(C).astype(np.int64), want)
    # K = 0: the zero matrix, or C unchanged when accumulating
    Z = dev(kind, C0)
    sr.semiring_mul(kind, Z, dev(kind, A[:, :0]), dev(kind, B[:0]), K=0)
    assert not host(Z).any()
    Z2 = dev(kind, C0)
    sr.semiring_mul(kind, Z2, dev(kind, A[:, :0]), dev(kind, B[:0]), K=0, flags=sr.SR_ACCUMULATE)
    assert np.array_equal(host(Z2), C0)


@pytest.mark.parametrize("kind", AD_KINDS)
def test_ad_mul_unpadded_strides(kind):
    """Row strides that are multiples of 16 bytes but not of the wide tile:
    the last column chunk takes the 8-column fallback."""
    gen = synthgen.generator(1002)
    R, K, N = 150, 77, 200
    per16 = 16 // np.dtype(np_dtype(kind)).itemsize
    lda = ((K + per16 - 1) // per16) * per16
    ldb = ((N + per16 - 1) // per16) * per16
    A = rand_antidist(R, K, kind, gen)
    B = rand_antidist(K, N, kind, gen)
    C = dev(kind, np.zeros((R, N), np_dtype(kind)), ld=ldb)
    sr.semiring_mul(kind, C, dev(kind, A, ld=lda), dev(kind, B, ld=ldb))
    assert np.array_equal(host(C).astype(np.int64), oracle.ad_mul(A, B, S_OF[kind]))


@pytest.mark.parametrize("kind", AD_KINDS)
@pytest.mark.parametrize("R,K,N", [(64, 1024, 64), (130, 700, 70), (1, 5000, 17),
                                   (200, 300, 1000), (65, 257, 33), (3, 256, 16)])
def test_ad_mul_split_inner(kind, R, K, N):
    """Few output tiles and a long inner dimension: the inner loop is split
    over the four waves of a workgroup (ragged splits, partial last column
    chunk), with and without accumulation."""
    gen = synthgen.generator(1100 + R + K + N)
    A = rand_antidist(R, K, kind, gen, p=0.05)
    B = rand_antidist(K, N, kind, gen, p=0.05)
    C = sr.empty(kind, R, N)
    sr.semiring_mul(kind, C, dev(kind, A), dev(kind, B))
    assert np.array_equal(host(C).astype(np.int64), oracle.ad_mul(A, B, S_OF[kind]))
    C0 = rand_antidist(R, N, kind, gen, p=0.5)
    Cd = dev(kind, C0)
    sr.semiring_mul(kind, Cd, dev(kind, A), dev(kind, B), flags=sr.SR_ACCUMULATE)
    assert np.array_equal(host(Cd).astype(np.int64), oracle.ad_mul(A, B, S_OF[kind], C=C0))


def test_ad_mul_padding_untouched():
    """Columns between N and ld belong to the caller and are not written."""
    kind = sr.SR_ANTIDIST_U16
    gen = synthgen.generator(1003)
    A = rand_antidist(40, 30, kind, gen)
    B = rand_antidist(30, 50, kind, gen)
    buf = torch.full((40, 64), 7, dtype=torch.uint16, device="cuda")
    sr.semiring_mul(kind, buf[:, :50], dev(kind, A), dev(kind, B))
    h = host(buf)
    assert (h[:, 50:] == 7).all()
    assert np.array_equal(h[:, :50].astype(np.int64), oracle.ad_mul(A, B, 65535))


def test_ad_mul_config2():
    """Two 1024 x 1024 uint16 random digraphs, p = 0.05,
    distances in [1, 1000], 1% near 65535."""
    A = synthgen.cfg_antidist(D=1024, which=0)
    B = synthgen.cfg_antidist(D=1024, which=1)
    kind = sr.SR_ANTIDIST_U16
    C = sr.empty(kind, 1024, 1024)
    sr.semiring_mul(kind, C, dev(kind, A[:, :1024]), dev(kind, B[:, :1024]))
    want = oracle.ad_mul(A[:, :1024], B[:, :1024], 65535)
    assert np.array_equal(host(C).astype(np.int64), want)


# ---------------------------------------------------------------------------
# anti-distance closure
# ---------------------------------------------------------------------------
CLO_SIZES = [1, 2, 37, 64, 127, 128, 129, 200, 255, 256, 300, 513]


@pytest.mark.parametrize("kind", AD_KINDS)
@pytest.mark.parametrize("D", CLO_SIZES)
def test_ad_closure(kind, D):
    gen = synthgen.generator(2000 + D)
    p = min(0.5, 4.0 / max(D, 1))
    A = rand_antidist(D, D, kind, gen, p=p, wmax=S_OF[kind] // 3)
    T = dev(kind, A)
    sr.closure(kind, T)
    want = oracle.ad_closure(A, S_OF[kind])
    assert np.array_equal(host(T).astype(np.int64), want)


@pytest.mark.parametrize("kind", AD_KINDS)
def test_ad_closure_unpadded_stride(kind):
    gen = synthgen.generator(2001)
    D = 300
    per16 = 16 // np.dtype(np_dtype(kind)).itemsize
    ld = ((D + per16 - 1) // per16) * per16
    A = rand_antidist(D, D, kind, gen, p=0.02, wmax=S_OF[kind] // 4)
    T = dev(kind, A, ld=ld)
    sr.closure(kind, T)
    assert np.array_equal(host(T).astype(np.int64), oracle.ad_closure(A, S_OF[kind]))


def test_ad_closure_saturation_cycle():
    """Directed cycle with unit distances: closed form, including saturation
    (uint8, D = 300 > S) on the diagonal and far entries."""
    for kind, D in ((sr.SR_ANTIDIST_U8, 300), (sr.SR_ANTIDIST_U16, 257)):
        S = S_OF[kind]
        A = np.zeros((D, D), np_dtype(kind))
        A[np.arange(D), (np.arange(D) + 1) % D] = S - 1
        T = dev(kind, A)
        sr.closure(kind, T)
        i = np.arange(D)[:, None]
        j = np.arange(D)[None, :]
        d = ((j - i - 1) % D) + 1
        want = np.where(d >= S, 0, S - np.minimum(d, S))
        assert np.array_equal(host(T).astype(np.int64), want)


def test_ad_closure_config2():
    """Closure of a D = 1024 uint16 random digraph with heavy edges."""
    A = synthgen.cfg_antidist(D=1024, which=0)[:, :1024]
    kind = sr.SR_ANTIDIST_U16
    T = dev(kind, A)
    sr.closure(kind, T)
    assert np.array_equal(host(T).astype(np.int64), oracle.ad_closure(A, 65535))


def test_ad_closure_u8_config4_style():
    """uint8 with distances in [1, 200] (saturation after two hops)."""
    gen = synthgen.generator(2002)
    D = 700
    rows, cols = synthgen.bernoulli_edges(D, 0.05, gen)
    w = gen.integers(1, 201, size=len(rows))
    A = synthgen.encode_antidist(D, rows, cols, w, np.uint8)
    T = dev(sr.SR_ANTIDIST_U8, A)
    sr.closure(sr.SR_ANTIDIST_U8, T)
    assert np.array_equal(host(T).astype(np.int64), oracle.ad_closure(A, 255))


def test_closure_equals_repeated_squaring_on_gpu():
    """Sec. II: closure(A) = A * (I (+) A)^(D'-1), D' >= D, the power by
    repeated squaring -- computed here with the GPU product only, compared
    with the GPU closure (cross-checks the two kernel families)."""
    kind = sr.SR_ANTIDIST_U16
    gen = synthgen.generator(2003)
    D = 150
    A = rand_antidist(D, D, kind, gen, p=0.02, wmax=20000)
    P = np.maximum(A, (np.eye(D, dtype=np.uint16) * 65535))
    dP = dev(kind, P)
    m = 1
    while m < D - 1:
        dQ = sr.empty(kind, D, D)
        sr.semiring_mul(kind, dQ, dP, dP)
        dP = dQ
        m *= 2
    dR = sr.empty(kind, D, D)
    sr.semiring_mul(kind, dR, dev(kind, A), dP)
    T = dev(kind, A)
    sr.closure(kind, T)
    assert np.array_equal(host(dR), host(T))


# ---------------------------------------------------------------------------
# Boolean
# ---------------------------------------------------------------------------
BOOL_SHAPES = [(1, 1, 1), (5, 70, 3), (64, 64, 64), (100, 200, 300), (257, 33, 1000),
               (300, 1100, 129),
               # few output tiles, long inner dimension (the inner bits split
               # over the waves of a workgroup): whole and ragged slices
               (256, 256, 256), (4096, 300, 256), (70, 4000, 64), (33, 129, 512)]


@pytest.mark.parametrize("R,K,N", BOOL_SHAPES)
def test_bool_mul(R, K, N):
    gen = synthgen.generator(3000 + R + K + N)
    A = rand_bits(R, K, gen, 0.05)
    B = rand_bits(K, N, gen, 0.05)
    Aw = synthgen.pack_bits(A, synthgen.aligned_ld_words(K))
    Bw = synthgen.pack_bits(B, synthgen.aligned_ld_words(N))
    C = sr.empty(sr.SR_BOOL, R, N)
    sr.semiring_mul(sr.SR_BOOL, C, dev(sr.SR_BOOL, Aw, cols=K), dev(sr.SR_BOOL, Bw, cols=N),
                    K=K, N=N)
    got = host(C)
    want = oracle.bool_mul_words(Aw, Bw, K, N)
    nw = (N + 63) // 64
    assert np.array_equal(got[:, :nw], want[:, :nw])
    assert synthgen.padding_bits_clear(got, N)


def test_bool_mul_accumulate():
    gen = synthgen.generator(3001)
    R, K, N = 90, 140, 200
    A, B, C0 = rand_bits(R, K, gen), rand_bits(K, N, gen), rand_bits(R, N, gen)
    ldw = synthgen.aligned_ld_words(N)
    Aw = synthgen.pack_bits(A, synthgen.aligned_ld_words(K))
    Bw = synthgen.pack_bits(B, ldw)
    Cw = synthgen.pack_bits(C0, ldw)
    C = dev(sr.SR_BOOL, Cw, cols=N)
    sr.semiring_mul(sr.SR_BOOL, C, dev(sr.SR_BOOL, Aw, cols=K), dev(sr.SR_BOOL, Bw, cols=N),
                    K=K, N=N, flags=sr.SR_ACCUMULATE)
    want = oracle.bool_mul_words(Aw, Bw, K, N, C=Cw)
    assert np.array_equal(host(C)[:, :4], want[:, :4])


def test_bool_config1():
    """Boolean 256 x 256, p = 0.02: A * A and the closure."""
    W = synthgen.cfg_bool256()
    A = dev(sr.SR_BOOL, W, cols=256)
    C = sr.empty(sr.SR_BOOL, 256, 256)
    sr.semiring_mul(sr.SR_BOOL, C, A, A, K=256, N=256)
    assert np.array_equal(host(C)[:, :4], oracle.bool_mul_words(W, W, 256, 256)[:, :4])
    sr.closure(sr.SR_BOOL, A, D=256)
    assert np.array_equal(host(A)[:, :4], oracle.bool_closure_words(W, 256)[:, :4])


@pytest.mark.parametrize("D", [1, 5, 63, 64, 65, 200, 256, 257, 300, 600, 1100])
def test_bool_closure(D):
    gen = synthgen.generator(3100 + D)
    A = rand_bits(D, D, gen, min(0.5, 1.5 / max(D, 1)))
    ldw = synthgen.aligned_ld_words(D)
    Aw = synthgen.pack_bits(A, ldw)
    T = dev(sr.SR_BOOL, Aw, cols=D)
    sr.closure(sr.SR_BOOL, T, D=D)
    got = host(T)
    want = oracle.bool_closure_words(Aw, D)
    nw = (D + 63) // 64
    assert np.array_equal(got[:, :nw], want[:, :nw])
    assert synthgen.padding_bits_clear(got, D)


@pytest.mark.parametrize("case", ["cycle", "descending", "ascending", "dense"])
@pytest.mark.parametrize("D", [64, 100, 130, 200, 256])
def test_bool_closure_pivot_tile(D, case):
    """Graphs of at most 256 vertices are one pivot tile: its four phases
    (each block's diagonal closed step by step, its other words as a product,
    the block applied to the other rows) on inputs whose paths cross every
    phase in the order the phases resolve last ('descending'), first
    ('ascending'), all ones ('cycle') and dense ones."""
    gen = synthgen.generator(3400 + D + len(case))
    if case == "cycle":
        order = gen.permutation(D)
        A = np.zeros((D, D), dtype=np.uint8)
        A[order, np.roll(order, -1)] = 1
    elif case == "descending":
        A = rand_bits(D, D, gen, 0.3 / D)
        A[np.arange(1, D), np.arange(D - 1)] = 1
    elif case == "ascending":
        A = rand_bits(D, D, gen, 0.3 / D)
        A[np.arange(D - 1), np.arange(1, D)] = 1
    else:
        A = rand_bits(D, D, gen, 0.3)
    ldw = synthgen.aligned_ld_words(D)
    Aw = synthgen.pack_bits(A, ldw)
    T = dev(sr.SR_BOOL, Aw, cols=D)
    sr.closure(sr.SR_BOOL, T, D=D)
    want = oracle.bool_closure_words(Aw, D)
    nw = (D + 63) // 64
    got = host(T)
    assert np.array_equal(got[:, :nw], want[:, :nw])
    assert synthgen.padding_bits_clear(got, D)


@pytest.mark.parametrize("path", [0, sr.SR_BOOL_BITWISE, sr.SR_BOOL_M4R, sr.SR_BOOL_MFMA])
@pytest.mark.parametrize("D", [769, 2100, 4100])
def test_bool_closure_lookahead_and_serial(D, path):
    """Sizes with several lookahead rounds and each word-chunk width (8 and
    16 words), with the bulk update by size, bit-sliced, or by the
    four-Russians tables: the overlapped schedule and the serial one give the
    oracle's bits."""
    gen = synthgen.generator(3200 + D)
    A = rand_bits(D, D, gen, 1.2 / D)
    ldw = synthgen.aligned_ld_words(D)
    Aw = synthgen.pack_bits(A, ldw)
    T = dev(sr.SR_BOOL, Aw, cols=D)
    T2 = sr.clone(T)
    sr.closure(sr.SR_BOOL, T, D=D, flags=path)
    sr.closure(sr.SR_BOOL, T2, D=D, flags=sr.SR_SERIAL_PHASES | path)
    want = oracle.bool_closure_words(Aw, D)
    nw = (D + 63) // 64
    got = host(T)
    assert np.array_equal(got[:, :nw], want[:, :nw])
    assert np.array_equal(host(T2)[:, :nw], want[:, :nw])
    assert synthgen.padding_bits_clear(got, D)


def test_bool_closure_matches_antidist_on_01():
    """Boolean closure = anti-distance closure of the {0, S} matrix / S."""
    gen = synthgen.generator(3002)
    D = 333
    A = rand_bits(D, D, gen, 0.004)
    T = dev(sr.SR_BOOL, synthgen.pack_bits(A, synthgen.aligned_ld_words(D)), cols=D)
    sr.closure(sr.SR_BOOL, T, D=D)
    U = dev(sr.SR_ANTIDIST_U16, (A.astype(np.uint16) * 65535))
    sr.closure(sr.SR_ANTIDIST_U16, U)
    assert np.array_equal(synthgen.unpack_bits(host(T), D).astype(np.int64) * 65535,
                          host(U).astype(np.int64))


# ---------------------------------------------------------------------------
# entrywise (+)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kind", AD_KINDS)
def test_add(kind):
    gen = synthgen.generator(4000)
    R, N = 77, 333
    A = rand_antidist(R, N, kind, gen, p=0.6)
    B = rand_antidist(R, N, kind, gen, p=0.6)
    C = sr.empty(kind, R, N)
    dA = dev(kind, A)
    sr.semiring_add(kind, C, dA, dev(kind, B))
    assert np.array_equal(host(C), np.maximum(A, B))
    sr.semiring_add(kind, dA, dA, dev(kind, B))  # in place
    assert np.array_equal(host(dA), np.maximum(A, B))


def test_add_bool():
    gen = synthgen.generator(4001)
    R, N = 50, 300
    A, B = rand_bits(R, N, gen), rand_bits(R, N, gen)
    ldw = synthgen.aligned_ld_words(N)
    C = sr.empty(sr.SR_BOOL, R, N)
    sr.semiring_add(sr.SR_BOOL, C, dev(sr.SR_BOOL, synthgen.pack_bits(A, ldw), cols=N),
                    dev(sr.SR_BOOL, synthgen.pack_bits(B, ldw), cols=N), N=N)
    assert np.array_equal(synthgen.unpack_bits(host(C), N), np.maximum(A, B))


# ---------------------------------------------------------------------------
# batched closure
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kind", AD_KINDS)
def test_closure_batched(kind):
    gen = synthgen.generator(5000 + kind)
    sizes = [1, 5, 32, 33, 64, 100, 128, 129, 200, 257, 300, 45, 600]
    mats = []
    for n in sizes:
        rows, cols = synthgen.bernoulli_edges(n, float(gen.uniform(0.01, 0.2)), gen)
        w = gen.integers(1, 201, size=len(rows))
        mats.append(synthgen.encode_antidist(n, rows, cols, w, np_dtype(kind)))
    devs = [dev(kind, m) for m in mats]
    sr.closure_batched(kind, devs)
    torch.cuda.synchronize()
    for m, d in zip(mats, devs):
        assert np.array_equal(host(d).astype(np.int64), oracle.ad_closure(m, S_OF[kind])), m.shape


def test_closure_batched_matches_solo():
    """Each graph closed in a batch equals the same graph closed alone."""
    kind = sr.SR_ANTIDIST_U16
    batch = synthgen.cfg_batch(count=40, nlo=32, nhi=400, seed=77)
    mats = [synthgen.encode_antidist(n, r, c, w, np.uint16) for n, r, c, w in batch]
    a = [dev(kind, m) for m in mats]
    b = [dev(kind, m) for m in mats]
    sr.closure_batched(kind, a)
    for t in b:
        sr.closure(kind, t)
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert np.array_equal(host(x), host(y))


@pytest.mark.parametrize("kind", AD_KINDS)
def test_closure_batched_ragged_rounds(kind):
    """Graphs with different round counts, ragged last blocks (1025, 130, 257)
    and an empty graph (D = 0) in one batch."""
    gen = synthgen.generator(5100 + kind)
    sizes = [130, 7, 1025, 1, 257, 256, 129, 3]
    mats = []
    for n in sizes:
        rows, cols = synthgen.bernoulli_edges(n, float(gen.uniform(0.005, 0.05)), gen)
        w = gen.integers(1, 201, size=len(rows))
        mats.append(synthgen.encode_antidist(n, rows, cols, w, np_dtype(kind)))
    devs = [dev(kind, m) for m in mats]
    spare = dev(kind, mats[3])  # a 1 x 1 matrix passed with D = 0: left as it is
    before = host(spare).copy()
    sr.closure_batched(kind, devs + [spare], Ds=sizes + [0])
    torch.cuda.synchronize()
    for m, d in zip(mats, devs):
        assert np.array_equal(host(d).astype(np.int64), oracle.ad_closure(m, S_OF[kind])), m.shape
    assert np.array_equal(host(spare), before)


@pytest.mark.parametrize("kind", AD_KINDS)
def test_closure_batched_arena(kind):
    """A batch held in one BatchArena: same bits as the list form, and the
    oracle on a sample."""
    batch = synthgen.cfg_batch(count=50, nlo=1, nhi=600, seed=91 + kind)
    mats = [synthgen.encode_antidist(n, r, c, w, np_dtype(kind)) for n, r, c, w in batch]
    arena = sr.BatchArena(kind, [m.shape[0] for m in mats])
    arena.load(mats)
    devs = [dev(kind, m) for m in mats]
    sr.closure_batched(kind, arena)
    sr.closure_batched(kind, devs)
    torch.cuda.synchronize()
    for i, d in enumerate(devs):
        assert torch.equal(arena.view(i), d), i
    for i in (0, 7, 23, 49):
        want = oracle.ad_closure(mats[i], S_OF[kind])
        assert np.array_equal(host(arena.view(i)).astype(np.int64), want), mats[i].shape


# ---------------------------------------------------------------------------
# Boolean product on the matrix cores (SR_BOOL_MFMA)
# ---------------------------------------------------------------------------
@pytest.fixture(params=["f4", "i8"])
def mfma_format(request, monkeypatch):
    """Operand format of the matrix-core path (4-bit floats or int8)."""
    monkeypatch.setenv("SR_MFMA_FORMAT", request.param)
    return request.param


@pytest.mark.parametrize("R,K,N", [(1, 1, 1), (5, 3, 7), (64, 64, 64), (65, 130, 129),
                                   (200, 37, 300), (257, 300, 513), (128, 1000, 256),
                                   (300, 9, 1100), (4, 0, 70), (70, 2049, 33)])
def test_bool_mul_mfma(mfma_format, R, K, N):
    """The matrix-core path in each operand format against the oracle."""
    test_bool_mul_paths(sr.SR_BOOL_MFMA, R, K, N)


@pytest.mark.parametrize("D", [257, 300, 513, 769, 2100, 4100])
def test_bool_closure_mfma(mfma_format, D):
    """The Boolean closure with its bulk update on the matrix cores, each
    operand format, overlapped and serial schedules, against the oracle."""
    test_bool_closure_lookahead_and_serial(D, sr.SR_BOOL_MFMA)


@pytest.mark.parametrize("case", ["cycle", "descending", "random"])
@pytest.mark.parametrize("D", [257, 512, 513, 1024, 1100, 2048, 2304, 3000])
def test_bool_closure_mfma_chains(mfma_format, D, case):
    """The closure with its bulk update on the matrix cores on inputs whose
    paths chain through every pivot block ('cycle': one cycle through a random
    order of all vertices, closure all ones; 'descending': i -> i - 1 plus
    sparse edges, the order the blocked loop resolves last) and on random
    ones; even and odd block counts, ragged last blocks; against the oracle,
    overlapped and serial schedules."""
    gen = synthgen.generator(3300 + D + len(case))
    if case == "cycle":
        order = gen.permutation(D)
        A = np.zeros((D, D), dtype=np.uint8)
        A[order, np.roll(order, -1)] = 1
    elif case == "descending":
        A = rand_bits(D, D, gen, 0.3 / D)
        A[np.arange(1, D), np.arange(D - 1)] = 1
    else:
        A = rand_bits(D, D, gen, 1.5 / D)
    ldw = synthgen.aligned_ld_words(D)
    Aw = synthgen.pack_bits(A, ldw)
    T = dev(sr.SR_BOOL, Aw, cols=D)
    T2 = sr.clone(T)
    sr.closure(sr.SR_BOOL, T, D=D, flags=sr.SR_BOOL_MFMA)
    sr.closure(sr.SR_BOOL, T2, D=D, flags=sr.SR_BOOL_MFMA | sr.SR_SERIAL_PHASES)
    want = oracle.bool_closure_words(Aw, D)
    nw = (D + 63) // 64
    got = host(T)
    assert np.array_equal(got[:, :nw], want[:, :nw])
    assert np.array_equal(host(T2)[:, :nw], want[:, :nw])
    assert synthgen.padding_bits_clear(got, D)


@pytest.mark.parametrize("path", [sr.SR_BOOL_MFMA, sr.SR_BOOL_M4R])
@pytest.mark.parametrize("R,K,N", [(1, 1, 1), (5, 3, 7), (64, 64, 64), (65, 130, 129),
                                   (200, 37, 300), (257, 300, 513), (128, 1000, 256),
                                   (300, 9, 1100), (4, 0, 70)])
def test_bool_mul_paths(path, R, K, N):
    """The matrix-core and four-Russians paths against the oracle."""
    gen = synthgen.generator(6000 + R + K + N)
    A = rand_bits(R, K, gen, 0.05)
    B = rand_bits(K, N, gen, 0.05)
    lda, ldb = synthgen.aligned_ld_words(K), synthgen.aligned_ld_words(N)
    Aw, Bw = synthgen.pack_bits(A, lda), synthgen.pack_bits(B, ldb)
    C = sr.empty(sr.SR_BOOL, R, N)
    sr.semiring_mul(sr.SR_BOOL, C, dev(sr.SR_BOOL, Aw, cols=K), dev(sr.SR_BOOL, Bw, cols=N),
                    K=K, N=N, flags=path)
    want = oracle.bool_mul_words(Aw, Bw, K, N)
    nw = (N + 63) // 64
    got = host(C)
    assert np.array_equal(got[:, :nw], want[:, :nw])
    assert synthgen.padding_bits_clear(got, N)


@pytest.mark.parametrize("path", [sr.SR_BOOL_MFMA, sr.SR_BOOL_M4R])
def test_bool_mul_paths_accumulate_and_dense(path, mfma_format):
    """Accumulate mode, and dense inputs (counts up to K) equal to the
    bitwise path."""
    gen = synthgen.generator(6100)
    R, K, N = 300, 700, 260
    for p in (0.02, 0.5):
        A = rand_bits(R, K, gen, p)
        B = rand_bits(K, N, gen, p)
        C0 = rand_bits(R, N, gen, 0.1)
        ldk, ldn = synthgen.aligned_ld_words(K), synthgen.aligned_ld_words(N)
        Aw, Bw, Cw = synthgen.pack_bits(A, ldk), synthgen.pack_bits(B, ldn), synthgen.pack_bits(C0, ldn)
        dA, dB = dev(sr.SR_BOOL, Aw, cols=K), dev(sr.SR_BOOL, Bw, cols=N)
        C1 = dev(sr.SR_BOOL, Cw, cols=N)
        C2 = dev(sr.SR_BOOL, Cw, cols=N)
        sr.semiring_mul(sr.SR_BOOL, C1, dA, dB, K=K, N=N, flags=path | sr.SR_ACCUMULATE)
        sr.semiring_mul(sr.SR_BOOL, C2, dA, dB, K=K, N=N, flags=sr.SR_ACCUMULATE)
        want = oracle.bool_mul_words(Aw, Bw, K, N, C=Cw)
        nw = (N + 63) // 64
        assert np.array_equal(host(C1)[:, :nw], want[:, :nw])
        assert torch.equal(C1, C2)


# ---------------------------------------------------------------------------
# distance matrices (min, saturating +), entrywise operations, reflexive
# ---------------------------------------------------------------------------
DIST_KINDS = [sr.SR_DISTANCE_U16, sr.SR_DISTANCE_U8]


@pytest.mark.parametrize("kind", DIST_KINDS)
@pytest.mark.parametrize("R,K,N", [(1, 1, 1), (3, 5, 2), (65, 130, 129), (200, 37, 300),
                                   (257, 8, 513)])
def test_dist_mul(kind, R, K, N):
    gen = synthgen.generator(7000 + R + K + N + kind)
    S = S_OF[kind]
    A = rand_dist(R, K, kind, gen, p=0.3)
    B = rand_dist(K, N, kind, gen, p=0.3)
    C = sr.empty(kind, R, N)
    sr.semiring_mul(kind, C, dev(kind, A), dev(kind, B))
    assert np.array_equal(host(C).astype(np.int64), oracle.dist_mul(A, B, S))
    C0 = rand_dist(R, N, kind, gen, p=0.5)
    Cd = dev(kind, C0)
    sr.semiring_mul(kind, Cd, dev(kind, A), dev(kind, B), flags=sr.SR_ACCUMULATE)
    assert np.array_equal(host(Cd).astype(np.int64), oracle.dist_mul(A, B, S, C=C0))


@pytest.mark.parametrize("kind", DIST_KINDS)
@pytest.mark.parametrize("D", [1, 2, 37, 129, 300, 513])
def test_dist_closure(kind, D):
    gen = synthgen.generator(7100 + D + kind)
    S = S_OF[kind]
    A = rand_dist(D, D, kind, gen, p=min(0.5, 3.0 / D), wmax=S // 4)
    T = dev(kind, A)
    sr.closure(kind, T)
    want = oracle.dist_closure(A, S)
    assert np.array_equal(host(T).astype(np.int64), want)
    T2 = dev(kind, A)
    sr.closure(kind, T2, flags=sr.SR_SERIAL_PHASES | sr.SR_REFLEXIVE)
    assert np.array_equal(host(T2).astype(np.int64), oracle.reflexive(want, 0))


@pytest.mark.parametrize("kind", AD_KINDS)
def test_reflexive_closure_antidist(kind):
    gen = synthgen.generator(7200 + kind)
    S = S_OF[kind]
    for D in (1, 130, 300):
        A = rand_antidist(D, D, kind, gen, p=min(0.5, 2.0 / D), wmax=S // 3)
        T = dev(kind, A)
        sr.closure(kind, T, flags=sr.SR_REFLEXIVE)
        want = oracle.reflexive(oracle.ad_closure(A, S), S)
        assert np.array_equal(host(T).astype(np.int64), want), D


def test_reflexive_closure_bool():
    gen = synthgen.generator(7300)
    for D in (1, 65, 300, 600):
        A = rand_bits(D, D, gen, min(0.5, 1.5 / D))
        ldw = synthgen.aligned_ld_words(D)
        Aw = synthgen.pack_bits(A, ldw)
        T = dev(sr.SR_BOOL, Aw, cols=D)
        sr.closure(sr.SR_BOOL, T, D=D, flags=sr.SR_REFLEXIVE)
        want = oracle.reflexive(oracle.bool_closure(A), 1)
        got = host(T)
        assert np.array_equal(synthgen.unpack_bits(got, D), want), D
        assert synthgen.padding_bits_clear(got, D)


@pytest.mark.parametrize("kind", AD_KINDS + DIST_KINDS)
@pytest.mark.parametrize("op,name", [(sr.SR_EW_AND, "and"), (sr.SR_EW_OR, "or"),
                                     (sr.SR_EW_XOR, "xor"), (sr.SR_EW_NOT, "not")])
def test_ewise(kind, op, name):
    gen = synthgen.generator(7400 + kind * 10 + op)
    S = S_OF[kind]
    R, N = 77, 333
    A = gen.integers(0, S + 1, size=(R, N)).astype(np_dtype(kind))
    B = gen.integers(0, S + 1, size=(R, N)).astype(np_dtype(kind))
    A[0, :3] = [0, S, S]
    B[0, :3] = [S, 0, S]
    C = sr.empty(kind, R, N)
    sr.semiring_ewise(kind, op, C, dev(kind, A), None if name == "not" else dev(kind, B))
    want = oracle.ewise(name, A, None if name == "not" else B, S)
    assert np.array_equal(host(C).astype(np.int64), want)
    # in place (C = A)
    Ad = dev(kind, A)
    sr.semiring_ewise(kind, op, Ad, Ad, None if name == "not" else dev(kind, B))
    assert np.array_equal(host(Ad).astype(np.int64), want)


@pytest.mark.parametrize("N", [1, 63, 64, 65, 200, 1000])
@pytest.mark.parametrize("op,name", [(sr.SR_EW_AND, "and"), (sr.SR_EW_OR, "or"),
                                     (sr.SR_EW_XOR, "xor"), (sr.SR_EW_NOT, "not")])
def test_ewise_bool(N, op, name):
    gen = synthgen.generator(7500 + N + op)
    R = 37
    ld = synthgen.aligned_ld_words(N)
    Aw = synthgen.pack_bits(rand_bits(R, N, gen, 0.5), ld)
    Bw = synthgen.pack_bits(rand_bits(R, N, gen, 0.5), ld)
    C = sr.empty(sr.SR_BOOL, R, N)
    sr.semiring_ewise(sr.SR_BOOL, op, C, dev(sr.SR_BOOL, Aw, cols=N),
                      None if name == "not" else dev(sr.SR_BOOL, Bw, cols=N), N=N)
    want = oracle.ewise_words(name, Aw, N, None if name == "not" else Bw)
    nw = (N + 63) // 64
    got = host(C)
    assert np.array_equal(got[:, :nw], want[:, :nw])
    assert synthgen.padding_bits_clear(got, N)


# operands above 16 MiB take the streaming (nontemporal) form of the kernel;
# ragged rows end in a partial 16-byte group
STREAM_SHAPES = {sr.SR_ANTIDIST_U8: (4200, 4001), sr.SR_ANTIDIST_U16: (2900, 3001),
                 sr.SR_ANTIDIST_U32: (2100, 2001), sr.SR_DISTANCE_U16: (2900, 3001)}


@pytest.mark.parametrize("kind", list(STREAM_SHAPES))
@pytest.mark.parametrize("op,name", [(sr.SR_EW_AND, "and"), (sr.SR_EW_OR, "or"),
                                     (sr.SR_EW_XOR, "xor"), (sr.SR_EW_NOT, "not")])
def test_ewise_streaming_sizes(kind, op, name):
    gen = synthgen.generator(7700 + kind * 10 + op)
    S = S_OF[kind]
    R, N = STREAM_SHAPES[kind]
    A = gen.integers(0, S + 1, size=(R, N)).astype(np_dtype(kind))
    B = gen.integers(0, S + 1, size=(R, N)).astype(np_dtype(kind))
    C = sr.empty(kind, R, N)
    sr.semiring_ewise(kind, op, C, dev(kind, A), None if name == "not" else dev(kind, B))
    want = oracle.ewise(name, A, None if name == "not" else B, S)
    assert np.array_equal(host(C).astype(np.int64), want)
    Ad = dev(kind, A)
    sr.semiring_ewise(kind, op, Ad, Ad, None if name == "not" else dev(kind, B))
    assert np.array_equal(host(Ad).astype(np.int64), want)


@pytest.mark.parametrize("R", [1023, 1024])
def test_ewise_streaming_threshold(R):
    """Rows of 8192 uint16 entries (16 KiB): 1023 rows stay one row under
    the 16 MiB operand size that switches to the streaming form, 1024 rows
    reach it; both give the oracle's result."""
    kind = sr.SR_ANTIDIST_U16
    gen = synthgen.generator(7900 + R)
    A = gen.integers(0, 65536, size=(R, 8192)).astype(np.uint16)
    B = gen.integers(0, 65536, size=(R, 8192)).astype(np.uint16)
    C = sr.empty(kind, R, 8192)
    sr.semiring_add(kind, C, dev(kind, A), dev(kind, B))
    assert np.array_equal(host(C).astype(np.int64), oracle.ewise("or", A, B))


@pytest.mark.parametrize("op,name", [(sr.SR_EW_AND, "and"), (sr.SR_EW_OR, "or"),
                                     (sr.SR_EW_XOR, "xor"), (sr.SR_EW_NOT, "not")])
def test_ewise_bool_streaming_size(op, name):
    gen = synthgen.generator(7800 + op)
    R, N = 1040, 130001          # 2032 words a row, 16 MiB and more per operand
    ld = synthgen.aligned_ld_words(N)
    Aw = synthgen.pack_bits(rand_bits(R, N, gen, 0.5), ld)
    Bw = synthgen.pack_bits(rand_bits(R, N, gen, 0.5), ld)
    C = sr.empty(sr.SR_BOOL, R, N)
    sr.semiring_ewise(sr.SR_BOOL, op, C, dev(sr.SR_BOOL, Aw, cols=N),
                      None if name == "not" else dev(sr.SR_BOOL, Bw, cols=N), N=N)
    want = oracle.ewise_words(name, Aw, N, None if name == "not" else Bw)
    nw = (N + 63) // 64
    got = host(C)
    assert np.array_equal(got[:, :nw], want[:, :nw])
    assert synthgen.padding_bits_clear(got, N)


@pytest.mark.parametrize("kind", DIST_KINDS)
def test_dist_add_is_min(kind):
    gen = synthgen.generator(7600 + kind)
    A = rand_dist(50, 70, kind, gen, p=0.5)
    B = rand_dist(50, 70, kind, gen, p=0.5)
    C = sr.empty(kind, 50, 70)
    sr.semiring_add(kind, C, dev(kind, A), dev(kind, B))
    assert np.array_equal(host(C).astype(np.int64), np.minimum(A, B).astype(np.int64))


@pytest.mark.parametrize("dense", [True, False])
@pytest.mark.parametrize("kind", [sr.SR_ANTIDIST_U8, sr.SR_DISTANCE_U8])
def test_closure_batched_u8_every_byte(kind, dense):
    """uint8 batches are widened by the first round's launches and narrowed
    by each graph's last-round launches: every byte value 0..255 on the way
    in (dense uniform bytes) and a wide spread of values on the way out
    (sparse uniform bytes), graphs of one to three rounds, against the
    oracle."""
    gen = synthgen.generator(7800 + kind + (10 if dense else 0))
    S = S_OF[kind]
    sizes = [1, 7, 64, 128, 129, 200, 300]
    mats = []
    for n in sizes:
        if dense:
            m = gen.integers(0, 256, size=(n, n)).astype(np.uint8)
        else:
            vals = gen.integers(0, 256, size=(n, n))
            m = np.where(gen.random((n, n)) < min(0.5, 2.0 / n), vals,
                         S if kind in DIST_KINDS else 0).astype(np.uint8)
        mats.append(m)
    if dense:
        assert len(np.unique(np.concatenate([m.ravel() for m in mats]))) == 256
    devs = [dev(kind, m) for m in mats]
    sr.closure_batched(kind, devs)
    for d, m in zip(devs, mats):
        want = oracle.dist_closure(m, S) if kind in DIST_KINDS else oracle.ad_closure(m, S)
        assert np.array_equal(host(d).astype(np.int64), want), m.shape


@pytest.mark.parametrize("kind", AD_KINDS + DIST_KINDS)
def test_closure_batched_dist_and_reflexive(kind):
    """Batches of distance matrices, and the reflexive flag, for all kinds."""
    gen = synthgen.generator(7700 + kind)
    S = S_OF[kind]
    sizes = [130, 7, 300, 1, 64]
    if kind in DIST_KINDS:
        mats = [rand_dist(n, n, kind, gen, p=min(0.5, 3.0 / n), wmax=S // 4) for n in sizes]
        want = [oracle.reflexive(oracle.dist_closure(m, S), 0) for m in mats]
    else:
        mats = [rand_antidist(n, n, kind, gen, p=min(0.5, 3.0 / n), wmax=S // 4) for n in sizes]
        want = [oracle.reflexive(oracle.ad_closure(m, S), S) for m in mats]
    devs = [dev(kind, m) for m in mats]
    sr.closure_batched(kind, devs, flags=sr.SR_REFLEXIVE)
    for d, w, m in zip(devs, want, mats):
        assert np.array_equal(host(d).astype(np.int64), w), m.shape
    plain = [dev(kind, m) for m in mats]
    sr.closure_batched(kind, plain)
    for d, m in zip(plain, mats):
        ref = oracle.dist_closure(m, S) if kind in DIST_KINDS else oracle.ad_closure(m, S)
        assert np.array_equal(host(d).astype(np.int64), ref), m.shape


# ---------------------------------------------------------------------------
# the two closure methods: blocked Warshall loop and repeated squaring
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kind", [sr.SR_ANTIDIST_U16, sr.SR_ANTIDIST_U8, sr.SR_DISTANCE_U16,
                                  sr.SR_ANTIDIST_U32, sr.SR_DISTANCE_U32, sr.SR_BOOL])
@pytest.mark.parametrize("D", [1, 2, 3, 130, 257, 700])
@pytest.mark.parametrize("method", [sr.SR_CLOSURE_SQUARING, sr.SR_CLOSURE_WARSHALL, 0])
def test_closure_methods(kind, D, method):
    """closure() forced to repeated squaring (eq. trcl), forced to the blocked
    loop, and by default (squaring for anti-distance and distance matrices of
    192..1024 vertices), each against the oracle; sizes with no squaring
    (D = 1, 2), one, and several, with ragged tiles; reflexive form too."""
    gen = synthgen.generator(9900 + 10 * kind + D)
    S = S_OF.get(kind, 1)
    if kind == sr.SR_BOOL:
        A = rand_bits(D, D, gen, min(0.5, 2.0 / D))
        ldw = synthgen.aligned_ld_words(D)
        T = dev(sr.SR_BOOL, synthgen.pack_bits(A, ldw), cols=D)
        want = oracle.bool_closure(A)
    elif kind in (sr.SR_DISTANCE_U16, sr.SR_DISTANCE_U32):
        A = rand_dist(D, D, kind, gen, p=min(0.5, 2.0 / D), wmax=S // 5)
        T = sr.to_device(kind, A)
        want = oracle.dist_closure(A, S)
    else:
        A = rand_antidist(D, D, kind, gen, p=min(0.5, 2.0 / D), wmax=S // 5)
        T = sr.to_device(kind, A)
        want = oracle.ad_closure(A, S)
    T2 = sr.clone(T)
    sr.closure(kind, T, D=D, flags=method)
    sr.closure(kind, T2, D=D, flags=method | sr.SR_REFLEXIVE)
    torch.cuda.synchronize()
    one = 1 if kind == sr.SR_BOOL else (0 if kind in (sr.SR_DISTANCE_U16, sr.SR_DISTANCE_U32)
                                         else S)
    if kind == sr.SR_BOOL:
        got, got2 = synthgen.unpack_bits(host(T), D), synthgen.unpack_bits(host(T2), D)
        assert synthgen.padding_bits_clear(host(T), D)
    else:
        got, got2 = host(T).astype(np.int64), host(T2).astype(np.int64)
    assert np.array_equal(got, want)
    assert np.array_equal(got2, oracle.reflexive(want, one))


def _squaring_input(case, kind, D, gen):
    """Inputs whose repeated squaring stops early or late: 'dense' (every
    edge, one weight: the first squaring leaves P unchanged), 'path' (a
    directed path 0 -> 1 -> ... of small weights plus random heavier edges
    from higher to lower vertices: best paths of D - 1 edges, so no squaring
    is skipped), 'random' (the 1024-vertex p = 0.05 generator: stops part way)."""
    S = S_OF[kind]
    if case == "dense":
        A = np.full((D, D), S - 3, dtype=np.int64)
        np.fill_diagonal(A, 0)
    elif case == "path":
        A = np.zeros((D, D), dtype=np.int64)
        for i in range(D - 1):
            A[i, i + 1] = S - 1
        back = gen.integers(0, D, size=(D, 2))
        for a, b in back:
            if a > b:
                A[a, b] = S - int(gen.integers(2, 50))
    elif kind == sr.SR_ANTIDIST_U8:
        A = synthgen.cfg_antidist_u8(D=D)[:, :D].astype(np.int64)
    else:
        # uint32: the same distances, entries S - w
        A = synthgen.cfg_antidist(D=D)[:, :D].astype(np.int64)
        A = np.where(A > 0, A + (S - 65535), 0)
    return A.astype(np_dtype(kind))


@pytest.mark.parametrize("kind", [sr.SR_ANTIDIST_U16, sr.SR_ANTIDIST_U8, sr.SR_ANTIDIST_U32,
                                  sr.SR_DISTANCE_U16])
@pytest.mark.parametrize("case", ["dense", "path", "random"])
def test_squaring_early_exit(kind, case):
    """The squaring closure skips, on the device, the squarings after one
    that left P unchanged; the result is the closure whether that happens
    after the first squaring, part way or never."""
    D = 700 if case == "path" else 1024
    gen = synthgen.generator(4242 + kind)
    S = S_OF[kind]
    A = _squaring_input(case, kind, D, gen)
    if kind == sr.SR_DISTANCE_U16:
        A = (S - A.astype(np.int64)).astype(np_dtype(kind))
        want = oracle.dist_closure(A, S)
    else:
        want = oracle.ad_closure(A, S)
    T = sr.to_device(kind, A)
    sr.closure(kind, T, D=D, flags=sr.SR_CLOSURE_SQUARING)
    assert np.array_equal(host(T).astype(np.int64), want)


@pytest.mark.parametrize("kind", [sr.SR_ANTIDIST_U16, sr.SR_ANTIDIST_U8, sr.SR_DISTANCE_U16,
                                  sr.SR_ANTIDIST_U32])
@pytest.mark.parametrize("D", [1024, 1100, 1537, 2100])
def test_closure_big_blocks(kind, D):
    """Mid sizes (above the whole-matrix squaring range): blocks of 512
    pivots, each closed by squaring, panels and update as products on blocks
    of the matrix (a ragged last block), against the oracle and against the
    forced blocked loop."""
    gen = synthgen.generator(9950 + 10 * kind + D)
    S = S_OF[kind]
    if kind == sr.SR_DISTANCE_U16:
        A = rand_dist(D, D, kind, gen, p=2.0 / D, wmax=S // 6)
        want = oracle.dist_closure(A, S)
    else:
        A = rand_antidist(D, D, kind, gen, p=2.0 / D, wmax=S // 6)
        want = oracle.ad_closure(A, S)
    T = sr.to_device(kind, A)
    T2 = sr.clone(T)
    sr.closure(kind, T)
    sr.closure(kind, T2, flags=sr.SR_CLOSURE_WARSHALL)
    torch.cuda.synchronize()
    assert np.array_equal(host(T).astype(np.int64), want)
    assert np.array_equal(host(T2).astype(np.int64), want)


@pytest.mark.parametrize("kind", [sr.SR_ANTIDIST_U16, sr.SR_ANTIDIST_U8, sr.SR_ANTIDIST_U32])
@pytest.mark.parametrize("B,D", [(256, 1024), (256, 1300), (768, 1024), (1024, 2000)])
def test_closure_big_blocks_tuned_block(kind, B, D, tmp_path):
    """Big pivot blocks of a tuned size (an autotuning entry loaded from its
    JSON file): with blocks of 256 a round's four panel products and four
    block products each share one launch; ragged last blocks take one
    launch per product.  Against the oracle."""
    gen = synthgen.generator(9970 + 10 * kind + B + D)
    S = S_OF[kind]
    A = rand_antidist(D, D, kind, gen, p=3.0 / D, wmax=S // 6)
    want = oracle.ad_closure(A, S)
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    cls = int(np.ceil(np.log2(D)))
    f = tmp_path / "tune.json"
    f.write_text('{"format": "libsemiring-autotune-1", "entries": [\n'
                 '{"arch": "%s", "op": 1, "kind": %d, "class": [%d, 0, 0], "choice": %d}\n]}\n'
                 % (arch, kind, cls, sr.SR_CLOSURE_BIG_BLOCKS | ((B // 64) << 16)))
    sr.autotune_clear()
    try:
        sr.autotune_load(str(f))
        T = sr.to_device(kind, A)
        sr.closure(kind, T)
        torch.cuda.synchronize()
        assert np.array_equal(host(T).astype(np.int64), want)
    finally:
        sr.autotune_clear()


@pytest.mark.parametrize("kind,D", [(sr.SR_ANTIDIST_U16, 3000), (sr.SR_ANTIDIST_U8, 4100),
                                    (sr.SR_DISTANCE_U16, 5000), (sr.SR_ANTIDIST_U16, 6144)])
def test_closure_loop_split_chain(kind, D):
    """The blocked loop at mid sizes, where the panels and the lookahead part
    run as K-split tiles: overlapped and serial schedules, every entry
    against the oracle's Warshall loop."""
    gen = synthgen.generator(9990 + kind + D)
    S = S_OF[kind]
    if kind == sr.SR_DISTANCE_U16:
        A = rand_dist(D, D, kind, gen, p=2.0 / D, wmax=S // 8)
        want = oracle.dist_closure(A, S)
    else:
        A = rand_antidist(D, D, kind, gen, p=2.0 / D, wmax=S // 8)
        want = oracle.ad_closure(A, S)
    T = sr.to_device(kind, A)
    T2 = sr.clone(T)
    sr.closure(kind, T, flags=sr.SR_CLOSURE_WARSHALL)
    sr.closure(kind, T2, flags=sr.SR_SERIAL_PHASES)
    torch.cuda.synchronize()
    assert np.array_equal(host(T).astype(np.int32), want)
    assert np.array_equal(host(T2).astype(np.int32), want)
