"""closure() captured into a HIP graph (torch.cuda.CUDAGraph) and replayed:
the fork onto the library's second stream and the join back are event-based,
so the whole lookahead schedule is captured.  Each replay runs on a fresh
input copied in eagerly, with eager library work between replays, and is
compared with the oracle."""
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
    torch.cuda.synchronize()


def _inputs(kind, D, n, seed):
    gen = synthgen.generator(seed)
    if kind == sr.SR_BOOL:
        ldw = synthgen.aligned_ld_words(D)
        mats = [rand_bits(D, D, gen, 2.0 / D) for _ in range(n)]
        return mats, [synthgen.pack_bits(m, ldw) for m in mats]
    if kind == sr.SR_DISTANCE_U16:
        mats = [rand_dist(D, D, kind, gen, p=2.0 / D, wmax=S_OF[kind] // 6) for _ in range(n)]
    else:
        mats = [rand_antidist(D, D, kind, gen, p=2.0 / D, wmax=S_OF[kind] // 6) for _ in range(n)]
    return mats, mats


def _want(kind, m):
    if kind == sr.SR_BOOL:
        return oracle.bool_closure(m)
    if kind == sr.SR_DISTANCE_U16:
        return oracle.dist_closure(m, S_OF[kind])
    return oracle.ad_closure(m, S_OF[kind])


def _got(kind, T, D):
    torch.cuda.synchronize()
    h = sr.to_host(T)
    if kind == sr.SR_BOOL:
        return synthgen.unpack_bits(h, D)
    return h.astype(np.int64)


@pytest.mark.parametrize("kind,D", [(sr.SR_ANTIDIST_U16, 700), (sr.SR_ANTIDIST_U32, 513),
                                    (sr.SR_DISTANCE_U16, 400), (sr.SR_BOOL, 1100)])
def test_closure_graph_replays(kind, D):
    mats, dev_fmt = _inputs(kind, D, 4, 9800 + kind + D)
    cols = D if kind == sr.SR_BOOL else None
    srcs = [sr.to_device(kind, h, cols=cols) for h in dev_fmt]
    T = sr.clone(srcs[0])
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    # an eager blocked-loop call on the capture stream first: the library's
    # second stream for it then exists before the capture starts (under
    # capture, closure() takes the blocked loop, which allocates nothing)
    with torch.cuda.stream(s):
        sr.closure(kind, T, D=D, flags=sr.SR_CLOSURE_WARSHALL)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        sr.closure(kind, T, D=D)
    torch.cuda.synchronize()
    other = sr.clone(srcs[1])
    for rep in range(3):
        i = rep + 1
        T.copy_(srcs[i])
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        want = _want(kind, mats[i])
        assert np.array_equal(_got(kind, T, D), want), "replay %d" % rep
        # eager library work between replays
        other.copy_(srcs[0])
        sr.closure(kind, other, D=D)
        torch.cuda.synchronize()
        want0 = _want(kind, mats[0])
        assert np.array_equal(_got(kind, other, D), want0), "eager after replay %d" % rep
