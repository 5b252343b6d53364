"""Pins for the oracle's distance-matrix dual, entrywise operations and
reflexive closure, and planted mistakes that the pins must catch.

The distance dual (the paper's section on distance matrices): entries 0..S
with S = no path, addition min, multiplication saturating +.  Its references
here are scipy / networkx shortest paths (library routines on an explicit
graph), brute-force relaxation, the
paper's De Morgan laws against the anti-distance oracle (a different function
with different arithmetic), and closed forms.  The entrywise operations
(table of Sec. V) are pinned by the laws the paper states (De Morgan),
involution, |a - b| = max - min, and their Boolean reduction; the reflexive
closure (eq. rtc) by paths of length zero allowed in scipy / networkx and by
repeated squaring of I (+) A.
"""
import networkx as nx
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import shortest_path

import oracle
import synthgen
from pins import rand_ad, rand_bool

SS = (255, 65535, 2 ** 32 - 1)


def rand_dist(R, C, S, gen, p=0.3, wmax=None):
    """Random distance matrix: present entries uniform in [0, wmax], absent = S."""
    wmax = S if wmax is None else wmax
    present = gen.random((R, C)) < p
    w = gen.integers(0, wmax + 1, size=(R, C))
    return np.where(present, np.minimum(w, S), S).astype(np.int64)


# ---------------------------------------------------------------------------
# independent references
# ---------------------------------------------------------------------------
def dist_product_shortest_path(A, B, S):
    """Two-edge shortest paths in the layered graph rows -> inner -> columns
    (scipy Dijkstra), saturated at S; weights shifted by +1 so that zero
    distances stay explicit edges (every path has exactly two edges)."""
    A = np.asarray(A, np.int64)
    B = np.asarray(B, np.int64)
    R, K = A.shape
    N = B.shape[1]
    ra, ka = np.nonzero(A < S)
    kb, nb = np.nonzero(B < S)
    src = np.concatenate([ra, R + kb])
    dst = np.concatenate([R + ka, R + K + nb])
    w = np.concatenate([A[ra, ka], B[kb, nb]]).astype(np.float64) + 1.0
    n = R + K + N
    G = sp.csr_matrix((w, (src, dst)), shape=(n, n))
    d = shortest_path(G, method="D", directed=True, indices=np.arange(R))[:, R + K:]
    d = np.where(np.isinf(d), np.inf, d - 2.0)
    return np.where(np.isinf(d), S, np.minimum(d, S)).astype(np.int64)


def dist_closure_networkx(A, S):
    """Minimum over walks of >= 1 edge: d+(i, j) = min_k w(i, k) + d(k, j),
    with d the ordinary shortest-path distance (d(k, k) = 0) from networkx's
    Dijkstra (which keeps explicit zero-weight edges), saturated at S."""
    A = np.asarray(A, np.int64)
    D = A.shape[0]
    dist = dict(nx.all_pairs_dijkstra_path_length(dist_graph(A, S), weight="weight"))
    out = np.full((D, D), S, np.int64)
    for a in range(D):
        for k in np.nonzero(A[a] < S)[0]:
            for b, dkb in dist[int(k)].items():
                out[a, b] = min(out[a, b], A[a, k] + dkb)
    return np.minimum(out, S)


def dist_graph(A, S):
    G = nx.DiGraph()
    G.add_nodes_from(range(A.shape[0]))
    for a, b in zip(*np.nonzero(A < S)):
        G.add_edge(int(a), int(b), weight=int(A[a, b]))
    return G


def dist_closure_bellman_ford(A, S):
    """Brute force: D rounds of relaxation over walks of >= 1 edge, in
    unbounded int64, saturated at the end."""
    A = np.asarray(A, np.int64)
    D = A.shape[0]
    INF = np.int64(1) << 40
    W = np.where(A < S, A, INF)
    d = W.copy()
    for _ in range(D):
        for k in range(D):
            d = np.minimum(d, d[:, k:k + 1] + W[k:k + 1, :])
    return np.minimum(d, S)


# ---------------------------------------------------------------------------
# pins (implementation passed in, so that mutants can be run through them)
# ---------------------------------------------------------------------------
def pin_dist_mul(mul, S, gen):
    for R, K, N in ((1, 1, 1), (3, 5, 2), (17, 9, 23), (30, 41, 12)):
        A = rand_dist(R, K, S, gen, p=0.4)
        B = rand_dist(K, N, S, gen, p=0.4)
        got = np.asarray(mul(A, B, S), np.int64)
        assert np.array_equal(got, dist_product_shortest_path(A, B, S)), (R, K, N)
        # De Morgan (distance section): not(A + B) = (not A) (x) (not B), the
        # right side by the anti-distance oracle
        assert np.array_equal(S - got, oracle.ad_mul(S - A, S - B, S)), (R, K, N)
    # K = 0: the additive zero (all S)
    assert np.array_equal(np.asarray(mul(np.zeros((3, 0), np.int64), np.zeros((0, 4), np.int64), S)),
                          np.full((3, 4), S))
    # the funny identity (0 on the diagonal, S elsewhere) is neutral
    A = rand_dist(9, 9, S, gen, p=0.5)
    I = np.where(np.eye(9, dtype=bool), 0, S)
    assert np.array_equal(np.asarray(mul(I, A, S)), A)
    assert np.array_equal(np.asarray(mul(A, I, S)), A)


def pin_dist_closure(clo, S, gen):
    for D in (1, 2, 5, 12, 23):
        for p in (0.15, 0.5):
            A = rand_dist(D, D, S, gen, p=p, wmax=S // 3)
            got = np.asarray(clo(A, S), np.int64)
            assert np.array_equal(got, dist_closure_bellman_ford(A, S)), (D, p)
    for D in (40, 70):
        A = rand_dist(D, D, S, gen, p=0.06, wmax=S // 4)
        got = np.asarray(clo(A, S), np.int64)
        assert np.array_equal(got, dist_closure_networkx(A, S)), D
        # De Morgan applied to every power: not dransclose(A) = transclose(not A)
        assert np.array_equal(S - got, oracle.ad_closure(S - A, S)), D
    # closed form: directed cycle with unit lengths, saturating when D >= S
    for D in (7, 300):
        if D > 60 and S > 255:
            continue
        A = np.full((D, D), S, np.int64)
        A[np.arange(D), (np.arange(D) + 1) % D] = 1
        i = np.arange(D)[:, None]
        j = np.arange(D)[None, :]
        want = np.minimum(((j - i - 1) % D) + 1, S)
        assert np.array_equal(np.asarray(clo(A, S), np.int64), want), D


def pin_ewise(ew, S, gen):
    A = gen.integers(0, S + 1, size=(23, 31))
    B = gen.integers(0, S + 1, size=(23, 31))
    A[0, :3] = [0, S, S]
    B[0, :3] = [S, 0, S]
    a_and, a_or = np.asarray(ew("and", A, B, S)), np.asarray(ew("or", A, B, S))
    a_xor, na = np.asarray(ew("xor", A, B, S)), np.asarray(ew("not", A, None, S))
    nb = np.asarray(ew("not", B, None, S))
    # De Morgan (distance section) and involution
    assert np.array_equal(S - a_or, np.asarray(ew("and", na, nb, S)))
    assert np.array_equal(S - a_and, np.asarray(ew("or", na, nb, S)))
    assert np.array_equal(np.asarray(ew("not", na, None, S)), A)
    # |a - b| is the larger minus the smaller
    assert np.array_equal(a_xor, a_or - a_and)
    assert (a_and <= A).all() and (a_and <= B).all() and (a_or >= A).all() and (a_or >= B).all()
    assert ((a_and == A) | (a_and == B)).all() and ((a_or == A) | (a_or == B)).all()
    # Boolean reduction: on {0, S} the operations are AND, OR, XOR, NOT times S
    P = rand_bool(17, 19, gen, 0.5).astype(bool)
    Q = rand_bool(17, 19, gen, 0.5).astype(bool)
    for op, f in (("and", np.logical_and), ("or", np.logical_or), ("xor", np.logical_xor)):
        assert np.array_equal(np.asarray(ew(op, P * S, Q * S, S)), f(P, Q) * S), op
    assert np.array_equal(np.asarray(ew("not", P * S, None, S)), np.logical_not(P) * S)


def pin_ewise_words(ew_words, gen):
    for N in (1, 63, 64, 65, 200):
        P = rand_bool(9, N, gen, 0.5)
        Q = rand_bool(9, N, gen, 0.5)
        ld = synthgen.aligned_ld_words(N)
        Pw, Qw = synthgen.pack_bits(P, ld), synthgen.pack_bits(Q, ld)
        for op, f in (("and", np.logical_and), ("or", np.logical_or), ("xor", np.logical_xor)):
            got = ew_words(op, Pw, N, Qw)
            assert np.array_equal(synthgen.unpack_bits(got, N), f(P, Q).astype(np.uint8)), (op, N)
            assert synthgen.padding_bits_clear(got, N)
        got = ew_words("not", Pw, N)
        assert np.array_equal(synthgen.unpack_bits(got, N), (1 - P).astype(np.uint8)), N
        assert synthgen.padding_bits_clear(got, N)


def pin_reflexive(refl, gen):
    # distance: shortest paths with the empty path allowed (d(i, i) = 0)
    S = 65535
    D = 30
    A = rand_dist(D, D, S, gen, p=0.1, wmax=1000)
    got = np.asarray(refl(oracle.dist_closure(A, S), 0))
    dist = dict(nx.all_pairs_dijkstra_path_length(dist_graph(A, S), weight="weight"))
    want = np.full((D, D), S, np.int64)
    for a in range(D):
        for b, v in dist[a].items():
            want[a, b] = min(v, S)
    assert np.array_equal(got, want)
    # anti-distance: I (+) T equals (I (+) A)^(D-1) by repeated squaring
    for S in SS:
        A = rand_ad(13, 13, S, gen, p=0.25)
        P = np.maximum(A, np.eye(13, dtype=np.int64) * S)
        Q = P.copy()
        for _ in range(4):  # (I + A)^16 >= paths of length <= 12
            Q = oracle.ad_mul(Q, Q, S)
        assert np.array_equal(np.asarray(refl(oracle.ad_closure(A, S), S)), Q), S
    # Boolean: networkx reflexive transitive closure
    B = rand_bool(25, 25, gen, 0.08)
    G = nx.DiGraph()
    G.add_nodes_from(range(25))
    G.add_edges_from(zip(*[x.tolist() for x in np.nonzero(B)]))
    H = nx.transitive_closure(G, reflexive=True)
    want = np.zeros((25, 25), np.uint8)
    for u, v in H.edges():
        want[u, v] = 1
    assert np.array_equal(np.asarray(refl(oracle.bool_closure(B), 1)), want)


# ---------------------------------------------------------------------------
# the oracle passes
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("S", SS)
def test_oracle_dist_mul(S):
    pin_dist_mul(oracle.dist_mul, S, np.random.default_rng(11))


@pytest.mark.parametrize("S", SS)
def test_oracle_dist_closure(S):
    pin_dist_closure(oracle.dist_closure, S, np.random.default_rng(12))


@pytest.mark.parametrize("S", SS + (1,))
def test_oracle_ewise(S):
    pin_ewise(oracle.ewise, S, np.random.default_rng(13))


def test_oracle_ewise_words():
    pin_ewise_words(oracle.ewise_words, np.random.default_rng(14))


def test_oracle_reflexive():
    pin_reflexive(oracle.reflexive, np.random.default_rng(15))


# ---------------------------------------------------------------------------
# planted mistakes must fail a pin
# ---------------------------------------------------------------------------
def _dist_mul_copy(A, B, S, init=None, times=None, better=np.minimum):
    A = np.asarray(A, np.int64)
    B = np.asarray(B, np.int64)
    times = times or (lambda a, b: np.minimum(a + b, S))
    P = np.full((A.shape[0], B.shape[1]), S if init is None else init, np.int64)
    for k in range(A.shape[1]):
        P = better(P, times(A[:, k:k + 1], B[k:k + 1, :]))
    return P


def _dist_clo_copy(A, S, times=None, kskip=0, reflexive_start=False):
    T = np.asarray(A, np.int64).copy()
    if reflexive_start:
        np.fill_diagonal(T, 0)
    times = times or (lambda a, b: np.minimum(a + b, S))
    for k in range(T.shape[0] - kskip):
        T = np.minimum(T, times(T[:, k:k + 1], T[k:k + 1, :]))
    return T


DIST_MUL_MUTANTS = {
    "init_zero": lambda A, B, S: _dist_mul_copy(A, B, S, init=0),
    "wraparound": lambda A, B, S: _dist_mul_copy(A, B, S, times=lambda a, b: (a + b) % (S + 1)),
    "max_not_min": lambda A, B, S: _dist_mul_copy(A, B, S, init=0, better=np.maximum),
    "off_by_one": lambda A, B, S: _dist_mul_copy(A, B, S, times=lambda a, b: np.minimum(a + b + 1, S)),
}

DIST_CLO_MUTANTS = {
    "skip_last_k": lambda A, S: _dist_clo_copy(A, S, kskip=1),
    # (dropping the saturation is not a mistake here: min with entries <= S
    # already bounds every value)
    "reflexive_start": lambda A, S: _dist_clo_copy(A, S, reflexive_start=True),
    "plain_min": lambda A, S: _dist_clo_copy(A, S, times=np.minimum),
}


def _ew_mutant(kind):
    def ew(op, A, B=None, S=None):
        A = np.asarray(A, np.int64)
        if kind == "xor_signed" and op == "xor":
            return A - np.asarray(B, np.int64)
        if kind == "not_off" and op == "not":
            return S - 1 - A
        if kind == "and_is_or" and op == "and":
            return np.maximum(A, np.asarray(B, np.int64))
        return oracle.ewise(op, A, B, S)
    return ew


def _refl_mutant(kind):
    def refl(T, one):
        out = np.array(T, copy=True)
        d = np.arange(min(out.shape))
        if kind == "always_max":
            out[d, d] = np.maximum(out[d, d], one)
        elif kind == "overwrite":
            out[d, d] = one if one else out[d, d]
        elif kind == "none":
            pass
        return out
    return refl


@pytest.mark.parametrize("name", sorted(DIST_MUL_MUTANTS))
def test_dist_mul_mutants_fail(name):
    with pytest.raises(AssertionError):
        for S in SS:
            pin_dist_mul(DIST_MUL_MUTANTS[name], S, np.random.default_rng(21))


@pytest.mark.parametrize("name", sorted(DIST_CLO_MUTANTS))
def test_dist_closure_mutants_fail(name):
    with pytest.raises(AssertionError):
        for S in SS:
            pin_dist_closure(DIST_CLO_MUTANTS[name], S, np.random.default_rng(22))


@pytest.mark.parametrize("name", ["xor_signed", "not_off", "and_is_or"])
def test_ewise_mutants_fail(name):
    with pytest.raises(AssertionError):
        for S in SS:
            pin_ewise(_ew_mutant(name), S, np.random.default_rng(23))


@pytest.mark.parametrize("name", ["always_max", "none"])
def test_reflexive_mutants_fail(name):
    with pytest.raises(AssertionError):
        pin_reflexive(_refl_mutant(name), np.random.default_rng(24))
