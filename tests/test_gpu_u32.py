"""Bit-exact parity of the 32-bit anti-distance and distance kinds
(S = 2^32 - 1) with the oracle's int64 loops, through the C ABI.

Sizes span several wave tiles (64 rows x 32 columns), pivot blocks of 128 and
ragged tails; strides include the 16-byte minimum (4 entries), which sends
the last columns of a row to the 4-column fallback tiles.
"""
import numpy as np
import pytest

import oracle
import paper_1705_08743_amd as sr
import synthgen
from gpu_util import rand_antidist, rand_dist, set_oracle_threads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

S = 2 ** 32 - 1
AD = sr.SR_ANTIDIST_U32
DI = sr.SR_DISTANCE_U32


@pytest.fixture(scope="module", autouse=True)
def _setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    set_oracle_threads()
    yield
    torch.cuda.synchronize()


def dev(host, ld=None):
    """Device copy; ld=None pads rows to 128 bytes, else exactly ld entries."""
    host = np.ascontiguousarray(host, dtype=np.uint32)
    if ld is None:
        return sr.to_device(AD, host)
    buf = torch.zeros((max(host.shape[0], 1), ld), dtype=torch.int32,
                      device="cuda").view(torch.uint32)
    buf[:host.shape[0], :host.shape[1]].copy_(torch.from_numpy(host))
    return buf[:host.shape[0], :host.shape[1]]


def host(t):
    torch.cuda.synchronize()
    return sr.to_host(t).astype(np.int64)


# (the K-split kernel takes those with a long inner loop and few tiles:
# 130 x 300 x 70, 512^3, 100 x 1000 x 37, 64 x 256 x 16, 1000 x 513 x 999)
MUL_SHAPES = [(1, 1, 1), (3, 5, 2), (64, 64, 64), (65, 130, 129), (200, 37, 300),
              (257, 8, 513), (130, 300, 70), (511, 129, 1000), (2100, 64, 2100),
              (512, 512, 512), (100, 1000, 37), (64, 256, 16), (1000, 513, 999)]


@pytest.mark.parametrize("R,K,N", MUL_SHAPES)
def test_ad32_mul(R, K, N):
    gen = synthgen.generator(9000 + R * 7 + K * 3 + N)
    A = rand_antidist(R, K, AD, gen, p=0.4)
    B = rand_antidist(K, N, AD, gen, p=0.4)
    C = sr.empty(AD, R, N)
    sr.semiring_mul(AD, C, dev(A), dev(B))
    assert np.array_equal(host(C), oracle.ad_mul(A, B, S))


def test_ad32_mul_accumulate_and_k0():
    gen = synthgen.generator(9001)
    for K in (45, 300):  # the second one on the K-split kernel
        A = rand_antidist(70, K, AD, gen)
        B = rand_antidist(K, 90, AD, gen)
        C0 = rand_antidist(70, 90, AD, gen, p=0.5)
        C = dev(C0)
        sr.semiring_mul(AD, C, dev(A), dev(B), flags=sr.SR_ACCUMULATE)
        assert np.array_equal(host(C), oracle.ad_mul(A, B, S, C=C0))
    Z = dev(C0)
    sr.semiring_mul(AD, Z, dev(A[:, :0]), dev(B[:0]), K=0)
    assert not host(Z).any()
    Z2 = dev(C0)
    sr.semiring_mul(AD, Z2, dev(A[:, :0]), dev(B[:0]), K=0, flags=sr.SR_ACCUMULATE)
    assert np.array_equal(host(Z2), C0.astype(np.int64))


@pytest.mark.parametrize("R,K,N", [(150, 77, 201), (70, 19, 30), (9, 3, 5)])
def test_ad32_mul_min_strides_and_padding(R, K, N):
    """Row strides of 16 bytes granularity (not multiples of the 32-column
    tile); the caller's columns between N and ld are left as they were."""
    gen = synthgen.generator(9002 + R)
    lda, ldb = -(-K // 4) * 4, -(-N // 4) * 4
    A = rand_antidist(R, K, AD, gen)
    B = rand_antidist(K, N, AD, gen)
    buf = torch.full((R, ldb + 4), 7, dtype=torch.int32, device="cuda").view(torch.uint32)
    sr.semiring_mul(AD, buf[:, :N], dev(A, ld=lda), dev(B, ld=ldb))
    full = host(buf)
    assert np.array_equal(full[:, :N], oracle.ad_mul(A, B, S))
    assert (full[:, N:] == 7).all()


CLO_SIZES = [1, 2, 37, 64, 127, 128, 129, 200, 255, 256, 300, 513, 1100]


@pytest.mark.parametrize("D", CLO_SIZES)
def test_ad32_closure(D):
    gen = synthgen.generator(9100 + D)
    A = rand_antidist(D, D, AD, gen, p=min(0.5, 4.0 / D), wmax=S // 3)
    T = dev(A)
    sr.closure(AD, T)
    assert np.array_equal(host(T), oracle.ad_closure(A, S))


@pytest.mark.parametrize("D", [769, 2100])
def test_ad32_closure_lookahead_and_serial(D):
    """Several lookahead rounds (second stream) and the serial schedule, both
    against the oracle; D = 2100 also has a partial last column chunk."""
    gen = synthgen.generator(9103 + D)
    A = rand_antidist(D, D, AD, gen, p=2.0 / D, wmax=S // 6)
    want = oracle.ad_closure(A, S)
    T = dev(A)
    sr.closure(AD, T)
    T2 = dev(A)
    sr.closure(AD, T2, flags=sr.SR_SERIAL_PHASES)
    assert np.array_equal(host(T), want)
    assert np.array_equal(host(T2), want)


@pytest.mark.parametrize("D", [130, 300])
def test_ad32_closure_min_stride(D):
    gen = synthgen.generator(9101 + D)
    A = rand_antidist(D, D, AD, gen, p=0.02, wmax=S // 4)
    T = dev(A, ld=-(-D // 4) * 4)
    sr.closure(AD, T)
    assert np.array_equal(host(T), oracle.ad_closure(A, S))


def test_ad32_closure_saturation_cycle():
    """Directed cycle whose edges have distance just over S/3: closed form,
    with paths of three or more edges saturating to 0 (no path)."""
    D = 257
    w = S // 3 + 1
    A = np.zeros((D, D), np.uint32)
    A[np.arange(D), (np.arange(D) + 1) % D] = S - w
    T = dev(A)
    sr.closure(AD, T)
    i = np.arange(D)[:, None]
    j = np.arange(D)[None, :]
    hops = ((j - i - 1) % D) + 1
    want = np.where(hops * w >= S, 0, S - np.minimum(hops * w, S))
    assert np.array_equal(host(T), want)


def test_ad32_closure_agrees_with_u16_on_scaled_input():
    """Entries S16 - w (uint16) and S32 - w (uint32) encode the same
    distances; with all path lengths below 65535 the two closures encode the
    same distances too (a cross-check of the 32-bit and 16-bit kernels)."""
    gen = synthgen.generator(9102)
    D = 700
    rows, cols = synthgen.bernoulli_edges(D, 0.01, gen)
    w = gen.integers(1, 60, size=len(rows))
    A16 = synthgen.encode_antidist(D, rows, cols, w, np.uint16)
    A32 = np.where(A16 > 0, S - (65535 - A16.astype(np.int64)), 0).astype(np.uint32)
    T16 = sr.to_device(sr.SR_ANTIDIST_U16, A16)
    T32 = dev(A32)
    sr.closure(sr.SR_ANTIDIST_U16, T16)
    sr.closure(AD, T32)
    h16 = host(T16)
    h32 = host(T32)
    d16 = np.where(h16 > 0, 65535 - h16, -1)
    d32 = np.where(h32 > 0, S - h32, -1)
    assert np.array_equal(d16, d32)


@pytest.mark.parametrize("R,K,N", [(1, 1, 1), (3, 5, 2), (65, 130, 129), (200, 37, 300)])
def test_dist32_mul(R, K, N):
    gen = synthgen.generator(9200 + R + K + N)
    A = rand_dist(R, K, DI, gen, p=0.3)
    B = rand_dist(K, N, DI, gen, p=0.3)
    C = sr.empty(DI, R, N)
    sr.semiring_mul(DI, C, dev(A), dev(B))
    assert np.array_equal(host(C), oracle.dist_mul(A, B, S))
    C0 = rand_dist(R, N, DI, gen, p=0.5)
    Cd = dev(C0)
    sr.semiring_mul(DI, Cd, dev(A), dev(B), flags=sr.SR_ACCUMULATE)
    assert np.array_equal(host(Cd), oracle.dist_mul(A, B, S, C=C0))


@pytest.mark.parametrize("D", [1, 37, 129, 300])
def test_dist32_closure_and_reflexive(D):
    gen = synthgen.generator(9300 + D)
    A = rand_dist(D, D, DI, gen, p=min(0.5, 3.0 / D), wmax=S // 4)
    T = dev(A)
    sr.closure(DI, T)
    want = oracle.dist_closure(A, S)
    assert np.array_equal(host(T), want)
    T2 = dev(A)
    sr.closure(DI, T2, flags=sr.SR_REFLEXIVE)
    assert np.array_equal(host(T2), oracle.reflexive(want, 0))


def test_ad32_reflexive():
    gen = synthgen.generator(9400)
    for D in (1, 130, 300):
        A = rand_antidist(D, D, AD, gen, p=min(0.5, 2.0 / D), wmax=S // 3)
        T = dev(A)
        sr.closure(AD, T, flags=sr.SR_REFLEXIVE)
        assert np.array_equal(host(T), oracle.reflexive(oracle.ad_closure(A, S), S)), D


@pytest.mark.parametrize("kind", [AD, DI])
@pytest.mark.parametrize("op,name", [(sr.SR_EW_AND, "and"), (sr.SR_EW_OR, "or"),
                                     (sr.SR_EW_XOR, "xor"), (sr.SR_EW_NOT, "not")])
def test_ewise32(kind, op, name):
    gen = synthgen.generator(9500 + kind * 10 + op)
    R, N = 77, 333
    A = gen.integers(0, S + 1, size=(R, N)).astype(np.uint32)
    B = gen.integers(0, S + 1, size=(R, N)).astype(np.uint32)
    A[0, :3] = [0, S, S]
    B[0, :3] = [S, 0, S]
    C = sr.empty(kind, R, N)
    sr.semiring_ewise(kind, op, C, dev(A), None if name == "not" else dev(B))
    want = oracle.ewise(name, A, None if name == "not" else B, S)
    assert np.array_equal(host(C), want)
    Ad = dev(A)
    sr.semiring_ewise(kind, op, Ad, Ad, None if name == "not" else dev(B))
    assert np.array_equal(host(Ad), want)


def test_add32():
    gen = synthgen.generator(9600)
    A = rand_antidist(50, 70, AD, gen, p=0.5)
    B = rand_antidist(50, 70, AD, gen, p=0.5)
    C = sr.empty(AD, 50, 70)
    sr.semiring_add(AD, C, dev(A), dev(B))
    assert np.array_equal(host(C), np.maximum(A, B).astype(np.int64))
    Cd = sr.empty(DI, 50, 70)
    sr.semiring_add(DI, Cd, dev(A), dev(B))
    assert np.array_equal(host(Cd), np.minimum(A, B).astype(np.int64))


@pytest.mark.parametrize("kind", [AD, sr.SR_DISTANCE_U32])
@pytest.mark.parametrize("flags", [0, sr.SR_REFLEXIVE])
def test_batched32(kind, flags):
    """32-bit batches (list form, and a prepared batch replayed from a
    captured graph on fresh contents): graphs of 0 to 1025 vertices with
    ragged tiles, against the oracle's int64 loops and the per-graph
    closure()."""
    sizes = [130, 7, 1025, 1, 257, 0, 64, 600, 383, 33]
    gen = synthgen.generator(9900 + kind + flags)

    def mats_for(seed):
        g = synthgen.generator(seed)
        out = []
        for n in sizes:
            p = min(0.5, float(g.uniform(1.0, 4.0)) / max(n, 1))
            out.append(rand_dist(n, n, kind, g, p=p, wmax=S // 7) if kind != AD
                       else rand_antidist(n, n, kind, g, p=p, wmax=S // 7))
        return out

    def want(m):
        w = oracle.dist_closure(m, S) if kind != AD else oracle.ad_closure(m, S)
        return oracle.reflexive(w, 0 if kind != AD else S) if flags else w

    mats = mats_for(int(gen.integers(1 << 30)))
    devs = [sr.to_device(kind, m) if m.shape[0] else sr.empty(kind, 0, 0) for m in mats]
    solo = [sr.clone(t) for t in devs]
    sr.closure_batched(kind, devs, Ds=sizes, flags=flags)
    for t, n in zip(solo, sizes):
        if n:
            sr.closure(kind, t, flags=flags)
    torch.cuda.synchronize()
    for t, s_, m in zip(devs, solo, mats):
        if m.shape[0]:
            assert np.array_equal(sr.to_host(t).astype(np.int64), want(m)), m.shape
            assert np.array_equal(sr.to_host(t), sr.to_host(s_)), m.shape
    # prepared and graph-captured
    sets = [mats_for(int(gen.integers(1 << 30))) for _ in range(2)]
    srcs = []
    for ms in sets:
        a = sr.BatchArena(kind, sizes)
        a.load(ms)
        srcs.append(a)
    work = sr.BatchArena(kind, sizes, zero=False)
    work.copy_(srcs[0])
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        pb = sr.PreparedBatch(kind, work, flags=flags)
        assert pb.autotune() == sr.SR_BATCH_TILE_64x32
        pb.run()
    torch.cuda.synchronize()
    for i, m in enumerate(sets[0]):
        if m.shape[0]:
            assert np.array_equal(sr.to_host(work.view(i)).astype(np.int64), want(m)), i
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        pb.run()
    work.copy_(srcs[1])
    torch.cuda.synchronize()
    g.replay()
    torch.cuda.synchronize()
    for i, m in enumerate(sets[1]):
        if m.shape[0]:
            assert np.array_equal(sr.to_host(work.view(i)).astype(np.int64), want(m)), i
    del g
    pb.close()
    sr.autotune_clear()


def test_ad32_closure_at_d4096():
    """D = 4096: the default (eight big pivot blocks of 512) and the forced
    128-pivot loop (32 rounds), every entry against the oracle's int64
    Warshall loop."""
    gen = synthgen.generator(9700)
    D = 4096
    A = rand_antidist(D, D, AD, gen, p=3.0 / D, wmax=S // 8)
    want = oracle.ad_closure(A, S)
    for flags in (0, sr.SR_CLOSURE_WARSHALL):
        T = dev(A)
        sr.closure(AD, T, flags=flags)
        assert np.array_equal(host(T), want), flags
