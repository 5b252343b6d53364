"""Prepared batches (sr_batch_create / sr_batch_run / sr_batch_autotune): the
batched closure of closure_batched with its plan built and uploaded once, so
that a closure of the whole batch is kernel launches only and can be captured
into a HIP graph.  Every update-tile shape, graph capture with replays on
fresh contents, the autotuner, the flags and degenerate batches, all against
the oracle bit for bit (integer arithmetic: tolerance 0)."""
import numpy as np
import pytest

import oracle
import paper_1705_08743_amd as sr
import synthgen
from gpu_util import S_OF, np_dtype, rand_antidist, rand_dist, set_oracle_threads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TILES = [sr.SR_BATCH_TILE_64x16, sr.SR_BATCH_TILE_64x32, sr.SR_BATCH_TILE_64x64]


@pytest.fixture(scope="module", autouse=True)
def _setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    set_oracle_threads()
    yield
    torch.cuda.synchronize()
    sr.autotune_clear()


def _mats(kind, sizes, seed):
    gen = synthgen.generator(seed)
    S = S_OF[kind]
    out = []
    for n in sizes:
        p = min(0.5, float(gen.uniform(1.0, 4.0)) / max(n, 1))
        if kind in (sr.SR_DISTANCE_U8, sr.SR_DISTANCE_U16):
            out.append(rand_dist(n, n, kind, gen, p=p, wmax=S // 5))
        else:
            out.append(rand_antidist(n, n, kind, gen, p=p, wmax=S // 5))
    return out


def _want(kind, m, reflexive=False):
    S = S_OF[kind]
    if kind in (sr.SR_DISTANCE_U8, sr.SR_DISTANCE_U16):
        w = oracle.dist_closure(m, S)
        return oracle.reflexive(w, 0) if reflexive else w
    w = oracle.ad_closure(m, S)
    return oracle.reflexive(w, S) if reflexive else w


def _host(t):
    torch.cuda.synchronize()
    return sr.to_host(t).astype(np.int64)


# graphs of 1 to 9 rounds of 128 pivots, ragged last blocks, an empty graph
SIZES = [130, 7, 1025, 1, 257, 256, 129, 3, 0, 64, 600, 383]


@pytest.mark.parametrize("kind", [sr.SR_ANTIDIST_U16, sr.SR_ANTIDIST_U8, sr.SR_DISTANCE_U16,
                                  sr.SR_DISTANCE_U8])
@pytest.mark.parametrize("tile", TILES)
def test_prepared_batch_each_tile(kind, tile):
    mats = _mats(kind, SIZES, 8800 + kind * 10 + tile)
    arena = sr.BatchArena(kind, SIZES)
    arena.load(mats)
    pb = sr.PreparedBatch(kind, arena, tile=tile)
    assert pb.tile == tile
    pb.run()
    for i, m in enumerate(mats):
        assert np.array_equal(_host(arena.view(i)), _want(kind, m)), (i, m.shape)
    # a second run closes the closed batch: the closure is idempotent
    pb.run()
    for i, m in enumerate(mats):
        assert np.array_equal(_host(arena.view(i)), _want(kind, m)), (i, m.shape)
    pb.close()


@pytest.mark.parametrize("kind", [sr.SR_ANTIDIST_U16, sr.SR_DISTANCE_U8])
def test_prepared_batch_reflexive(kind):
    mats = _mats(kind, SIZES, 8900 + kind)
    arena = sr.BatchArena(kind, SIZES)
    arena.load(mats)
    pb = sr.PreparedBatch(kind, arena, flags=sr.SR_REFLEXIVE)
    pb.run()
    for i, m in enumerate(mats):
        assert np.array_equal(_host(arena.view(i)), _want(kind, m, True)), (i, m.shape)
    pb.close()


def test_prepared_batch_degenerate():
    kind = sr.SR_ANTIDIST_U16
    empty = sr.BatchArena(kind, [])
    pb = sr.PreparedBatch(kind, empty)
    pb.run()
    assert pb.autotune() in (sr.SR_BATCH_TILE_AUTO,) + tuple(TILES)
    pb.close()
    zeros = sr.BatchArena(kind, [0, 0, 1])
    m = [np.zeros((0, 0), np.uint16), np.zeros((0, 0), np.uint16),
         np.array([[7]], dtype=np.uint16)]
    zeros.load(m)
    pb = sr.PreparedBatch(kind, zeros)
    pb.run()
    assert _host(zeros.view(2))[0, 0] == 7
    pb.close()
    with pytest.raises(ValueError):
        pb.run()


@pytest.mark.parametrize("kind", [sr.SR_ANTIDIST_U16, sr.SR_ANTIDIST_U8])
def test_prepared_batch_graph_replays(kind):
    """run() captured into a graph; three replays on fresh contents copied in
    eagerly, with eager closure_batched work between the replays; every
    replay and every eager call against the oracle."""
    batch = synthgen.cfg_batch(count=60, nlo=1, nhi=700, seed=4400 + kind)
    sets = []
    for r in range(4):
        gen = synthgen.generator(4500 + 10 * kind + r)
        mats = []
        for n, _, _, _ in batch:
            rows, cols = synthgen.bernoulli_edges(n, float(gen.uniform(0.005, 0.1)), gen)
            w = gen.integers(1, 201, size=len(rows))
            mats.append(synthgen.encode_antidist(n, rows, cols, w, np_dtype(kind)))
        sets.append(mats)
    sizes = [n for n, _, _, _ in batch]
    srcs = []
    for mats in sets:
        a = sr.BatchArena(kind, sizes)
        a.load(mats)
        srcs.append(a)
    work = sr.BatchArena(kind, sizes, zero=False)
    work.copy_(srcs[0])
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        pb = sr.PreparedBatch(kind, work)
        pb.run()  # eager run on the capture stream first
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        pb.run()
    torch.cuda.synchronize()
    other = sr.BatchArena(kind, sizes, zero=False)
    check = [0, 1, 17, 30, 59]
    for rep in range(3):
        i = rep + 1
        work.copy_(srcs[i])
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for j in check:
            want = oracle.ad_closure(sets[i][j], S_OF[kind])
            assert np.array_equal(_host(work.view(j)), want), ("replay", rep, j)
        other.copy_(srcs[0])
        sr.closure_batched(kind, other)
        torch.cuda.synchronize()
        for j in check:
            want = oracle.ad_closure(sets[0][j], S_OF[kind])
            assert np.array_equal(_host(other.view(j)), want), ("eager", rep, j)
        # the replay and the list form agree on every graph
        eager = sr.BatchArena(kind, sizes, zero=False)
        eager.copy_(srcs[i])
        sr.closure_batched(kind, eager)
        torch.cuda.synchronize()
        assert torch.equal(eager.buf, work.buf), rep
    del g
    pb.close()


@pytest.mark.parametrize("kind", [sr.SR_ANTIDIST_U16, sr.SR_ANTIDIST_U8])
def test_prepared_batch_graph_survives_autotune(kind):
    """A graph captured from a run with the 64 x 16 tiles, then the autotuner
    (which re-plans the handle for its pick): replaying the old graph on fresh
    contents still gives the oracle's closure, and so does a run with the new
    plan."""
    sizes = [int(n) for n, _, _, _ in synthgen.cfg_batch(count=70, nlo=8, nhi=800,
                                                            seed=5500 + kind)]
    sets = [_mats(kind, sizes, 5600 + 10 * kind + r) for r in range(3)]
    srcs = []
    for mats in sets:
        a = sr.BatchArena(kind, sizes)
        a.load(mats)
        srcs.append(a)
    work = sr.BatchArena(kind, sizes, zero=False)
    work.copy_(srcs[0])
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        pb = sr.PreparedBatch(kind, work, tile=sr.SR_BATCH_TILE_64x16)
        pb.run()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        pb.run()
    torch.cuda.synchronize()
    t = pb.autotune()
    torch.cuda.synchronize()
    assert t in TILES and pb.tile == t
    check = [0, 3, 33, 69]
    work.copy_(srcs[1])
    torch.cuda.synchronize()
    g.replay()
    torch.cuda.synchronize()
    for j in check:
        assert np.array_equal(_host(work.view(j)), _want(kind, sets[1][j])), ("replay", j)
    eager = sr.BatchArena(kind, sizes, zero=False)
    eager.copy_(srcs[1])
    sr.closure_batched(kind, eager)
    torch.cuda.synchronize()
    assert torch.equal(eager.buf, work.buf)
    work.copy_(srcs[2])
    pb.run()
    torch.cuda.synchronize()
    for j in check:
        assert np.array_equal(_host(work.view(j)), _want(kind, sets[2][j])), ("new plan", j)
    del g
    pb.close()
    sr.autotune_clear()


@pytest.mark.parametrize("kind", [sr.SR_ANTIDIST_U16, sr.SR_ANTIDIST_U8])
def test_prepared_batch_autotune(kind):
    """The autotuner picks one of the tile shapes, leaves the batch's
    matrices untouched, and the batch closes the same afterwards, as does
    closure_batched (which now takes the tuned shape for the class)."""
    sizes = [int(n) for n, _, _, _ in synthgen.cfg_batch(count=80, nlo=16, nhi=900,
                                                            seed=77 + kind)]
    mats = _mats(kind, sizes, 9100 + kind)
    arena = sr.BatchArena(kind, sizes)
    arena.load(mats)
    before = arena.buf.clone()
    pb = sr.PreparedBatch(kind, arena)
    t = pb.autotune()
    torch.cuda.synchronize()
    assert t in TILES and pb.tile == t
    assert torch.equal(arena.buf, before)
    pb.run()
    listed = [sr.to_device(kind, m) for m in mats]
    sr.closure_batched(kind, listed)
    torch.cuda.synchronize()
    for i in range(len(mats)):
        assert torch.equal(arena.view(i), listed[i]), i
    for i in (0, 5, 40, 79):
        assert np.array_equal(_host(arena.view(i)), _want(kind, mats[i])), mats[i].shape
    pb.close()
    sr.autotune_clear()


def test_prepared_batch_config4_sample():
    """4096 graphs (log-uniform sizes in [32, 1024]) through
    the prepared, graph-captured form: every graph equal to closure_batched,
    a sample against the oracle."""
    kind = sr.SR_ANTIDIST_U16
    batch = synthgen.cfg_batch()
    mats = [synthgen.encode_antidist(n, r, c, w, np.uint16) for n, r, c, w in batch]
    sizes = [m.shape[0] for m in mats]
    src = sr.BatchArena(kind, sizes)
    src.load(mats)
    work = sr.BatchArena(kind, sizes, zero=False)
    work.copy_(src)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        pb = sr.PreparedBatch(kind, work)
        pb.autotune()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        pb.run()
    torch.cuda.synchronize()
    work.copy_(src)
    torch.cuda.synchronize()
    g.replay()
    ref = sr.BatchArena(kind, sizes, zero=False)
    ref.copy_(src)
    sr.closure_batched(kind, ref)
    torch.cuda.synchronize()
    assert torch.equal(ref.buf, work.buf)
    idx = np.argsort(sizes)
    for i in list(idx[:2]) + list(idx[-2:]) + [int(idx[len(idx) // 2])]:
        want = oracle.ad_closure(mats[i], 65535)
        assert np.array_equal(_host(work.view(int(i))), want), mats[i].shape
    del g
    pb.close()
    sr.autotune_clear()


# ---------------------------------------------------------------------------
# Boolean batches: closed as {0, 255} anti-distance matrices in binary16
# working copies, packed back to bits
# ---------------------------------------------------------------------------
BOOL_SIZES = [130, 7, 1025, 1, 257, 256, 129, 3, 0, 64, 600, 383, 65, 63]


def _bool_mats(sizes, seed):
    from gpu_util import rand_bits
    gen = synthgen.generator(seed)
    return [rand_bits(n, n, gen, min(0.5, float(gen.uniform(0.5, 3.0)) / max(n, 1)))
            for n in sizes]


def _bool_got(t, n):
    h = sr.to_host(t)
    assert synthgen.padding_bits_clear(h, n)
    return synthgen.unpack_bits(h, n)


@pytest.mark.parametrize("flags", [0, sr.SR_REFLEXIVE])
def test_closure_batched_boolean(flags):
    """closure_batched on bit-packed matrices: the oracle's Boolean closure
    (and its reflexive form), padding bits kept clear, and the same bits as
    closure() of each graph on its own (the bit-sliced kernels)."""
    mats = _bool_mats(BOOL_SIZES, 6100 + flags)
    devs, solo = [], []
    for m in mats:
        n = m.shape[0]
        words = synthgen.pack_bits(m, synthgen.aligned_ld_words(max(n, 1)))
        devs.append(sr.to_device(sr.SR_BOOL, words, cols=max(n, 1))[:n])
        solo.append(sr.clone(devs[-1]))
    sr.closure_batched(sr.SR_BOOL, devs, Ds=BOOL_SIZES, flags=flags)
    for t, n in zip(solo, BOOL_SIZES):
        if n:
            sr.closure(sr.SR_BOOL, t, D=n, flags=flags)
    torch.cuda.synchronize()
    for t, s_, m in zip(devs, solo, mats):
        n = m.shape[0]
        if n == 0:
            continue
        want = oracle.bool_closure(m)
        if flags & sr.SR_REFLEXIVE:
            want = oracle.reflexive(want, 1)
        assert np.array_equal(_bool_got(t, n), want), n
        assert torch.equal(t, s_), n


@pytest.mark.parametrize("case", ["cycle", "descending", "ascending", "random"])
def test_closure_batched_boolean_small_phases(case):
    """Boolean graphs of at most 1024 vertices are closed in place, one
    workgroup each: every size class (up to 64, 128, 256, 512, 768, 1024
    vertices) with ragged sizes, on paths through all vertices in descending
    order (the order Warshall's loop resolves last), ascending order, one
    cycle (closure all ones) and random graphs; against the oracle."""
    sizes = [1024, 1000, 769, 700, 513, 300, 257, 200, 129, 100, 65, 64, 33, 2]
    gen = synthgen.generator(6300 + len(case))
    from gpu_util import rand_bits
    mats = []
    for n in sizes:
        if case == "cycle":
            order = gen.permutation(n)
            m = np.zeros((n, n), dtype=np.uint8)
            m[order, np.roll(order, -1)] = 1
        elif case == "descending":
            m = rand_bits(n, n, gen, 0.3 / n)
            m[np.arange(1, n), np.arange(n - 1)] = 1
        elif case == "ascending":
            m = rand_bits(n, n, gen, 0.3 / n)
            m[np.arange(n - 1), np.arange(1, n)] = 1
        else:
            m = rand_bits(n, n, gen, 1.5 / n)
        mats.append(m)
    devs = []
    for m in mats:
        n = m.shape[0]
        words = synthgen.pack_bits(m, synthgen.aligned_ld_words(n))
        devs.append(sr.to_device(sr.SR_BOOL, words, cols=n)[:n])
    sr.closure_batched(sr.SR_BOOL, devs, Ds=sizes)
    torch.cuda.synchronize()
    for t, m in zip(devs, mats):
        assert np.array_equal(_bool_got(t, m.shape[0]), oracle.bool_closure(m)), m.shape[0]


@pytest.mark.parametrize("tile", TILES)
def test_prepared_batch_boolean(tile):
    """A prepared Boolean batch with each update-tile shape, run eagerly and
    replayed from a captured graph on fresh contents."""
    sizes = BOOL_SIZES
    sets = [_bool_mats(sizes, 6200 + 10 * tile + r) for r in range(3)]
    packed = [[synthgen.pack_bits(m, max(2, -(-(-(-m.shape[0] // 64)) // 2) * 2)) for m in ms]
              for ms in sets]
    srcs = []
    for ps in packed:
        a = sr.BatchArena(sr.SR_BOOL, sizes)
        a.load(ps)
        srcs.append(a)
    work = sr.BatchArena(sr.SR_BOOL, sizes, zero=False)
    work.copy_(srcs[0])
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        pb = sr.PreparedBatch(sr.SR_BOOL, work, tile=tile)
        if tile == sr.SR_BATCH_TILE_64x64:
            # the autotuner on a Boolean batch leaves its matrices untouched
            before = work.buf.clone()
            assert pb.autotune() in TILES
            assert torch.equal(work.buf, before)
        pb.run()
    torch.cuda.synchronize()
    for i, m in enumerate(sets[0]):
        if m.shape[0]:
            assert np.array_equal(_bool_got(work.view(i), m.shape[0]), oracle.bool_closure(m))
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        pb.run()
    torch.cuda.synchronize()
    for r in (1, 2):
        work.copy_(srcs[r])
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for i, m in enumerate(sets[r]):
            if m.shape[0]:
                assert np.array_equal(_bool_got(work.view(i), m.shape[0]),
                                      oracle.bool_closure(m)), (r, i)
    del g
    pb.close()
