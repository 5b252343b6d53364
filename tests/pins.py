"""Independent checks ("pins") for the oracle.

Each pin compares an implementation of the product or the closure with
something that shares no code with it: a library routine (integer matmul,
scipy / networkx shortest paths and reachability), a brute force written here,
a closed form, or an algebraic law stated in the paper.  The pins take the
implementation as an argument so that the mutant tests can show that planted
mistakes are caught.

Conventions: anti-distance matrices are integer arrays with entries 0..S
(entry = S - distance, 0 = no edge; Sec. III and Sec. IV); Boolean matrices
are 0/1 arrays (Sec. II), entry (i, j) = edge i -> j.
"""
import math

import networkx as nx
import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import shortest_path

import synthgen

INF = np.int64(1) << 40


# ---------------------------------------------------------------------------
# independent references
# ---------------------------------------------------------------------------
def bool_product_matmul(A, B):
    """Boolean product via ordinary integer matrix multiplication: the count
    of k with A_ik = B_kj = 1 is positive iff (A*B)_ij = 1."""
    return (np.asarray(A, np.int64) @ np.asarray(B, np.int64) > 0).astype(np.uint8)


def ad_product_demorgan(A, B, S):
    """Anti-distance product through its De Morgan dual (Sec. IV):
    not(A * B) = (not A) + (not B) with not a = S - a and + the min-plus
    product of distances, saturated at S."""
    dA = S - np.asarray(A, np.int64)
    dB = S - np.asarray(B, np.int64)
    d = np.min(dA[:, :, None] + dB[None, :, :], axis=1) if A.shape[1] else \
        np.full((A.shape[0], B.shape[1]), S, np.int64)
    return S - np.minimum(d, S)


def ad_product_shortest_path(A, B, S):
    """Anti-distance product as two-edge shortest paths in a layered graph
    (rows of A -> inner index -> columns of B) solved by scipy's Dijkstra.
    Every edge weight is shifted by +1 (all paths have exactly two edges, so
    the shift adds exactly 2), which keeps zero distances as explicit edges."""
    A = np.asarray(A, np.int64)
    B = np.asarray(B, np.int64)
    R, K = A.shape
    N = B.shape[1]
    n = R + K + N
    ra, ka = np.nonzero(A > 0)
    kb, nb = np.nonzero(B > 0)
    src = np.concatenate([ra, R + kb])
    dst = np.concatenate([R + ka, R + K + nb])
    w = np.concatenate([S - A[ra, ka], S - B[kb, nb]]).astype(np.float64) + 1.0
    G = sp.csr_matrix((w, (src, dst)), shape=(n, n))
    dist = shortest_path(G, method="D", directed=True, indices=np.arange(R))
    d = dist[:, R + K:]
    out = np.zeros((R, N), np.int64)
    fin = np.isfinite(d)
    dd = np.rint(d[fin]).astype(np.int64) - 2
    out[fin] = np.where(dd >= S, 0, S - dd)
    return out


def bool_closure_bfs(A):
    """Brute-force reachability by breadth-first search from each vertex,
    seeded with its out-neighbours (paths of at least one edge)."""
    A = np.asarray(A, np.uint8)
    D = A.shape[0]
    out = np.zeros((D, D), np.uint8)
    for s in range(D):
        seen = np.zeros(D, bool)
        frontier = list(np.nonzero(A[s])[0])
        for v in frontier:
            seen[v] = True
        while frontier:
            nxt = []
            for u in frontier:
                for v in np.nonzero(A[u])[0]:
                    if not seen[v]:
                        seen[v] = True
                        nxt.append(v)
            frontier = nxt
        out[s] = seen
    return out


def bool_closure_networkx(A):
    A = np.asarray(A, np.uint8)
    D = A.shape[0]
    G = nx.DiGraph()
    G.add_nodes_from(range(D))
    G.add_edges_from(zip(*np.nonzero(A)))
    H = nx.transitive_closure(G, reflexive=False)
    out = np.zeros((D, D), np.uint8)
    for u, v in H.edges():
        out[u, v] = 1
    return out


def ad_closure_bellman_ford(A, S):
    """Brute force: shortest walk distances with >= 1 edge by repeated
    relaxation in unbounded int64 (D rounds cover every simple path and
    simple cycle), saturated at S only at the end."""
    A = np.asarray(A, np.int64)
    D = A.shape[0]
    W = np.where(A > 0, S - A, INF)
    d = W.copy()
    for _ in range(D):
        for k in range(D):
            cand = d[:, k:k + 1] + W[k:k + 1, :]
            d = np.minimum(d, cand)
    return np.where(d >= S, 0, S - np.minimum(d, S))


def ad_closure_networkx(A, S):
    """Closure via networkx Dijkstra: d+(i, j) = min over edges i -> k of
    w(i, k) + d(k, j), with d the ordinary shortest-path distance."""
    A = np.asarray(A, np.int64)
    D = A.shape[0]
    G = nx.DiGraph()
    G.add_nodes_from(range(D))
    for i, j in zip(*np.nonzero(A)):
        G.add_edge(int(i), int(j), weight=int(S - A[i, j]))
    dist = dict(nx.all_pairs_dijkstra_path_length(G, weight="weight"))
    out = np.zeros((D, D), np.int64)
    for i in range(D):
        best = np.full(D, INF)
        for k in np.nonzero(A[i])[0]:
            wik = S - A[i, k]
            for j, dkj in dist[int(k)].items():
                best[j] = min(best[j], wik + dkj)
        out[i] = np.where(best >= S, 0, S - np.minimum(best, S))
    return out


# ---------------------------------------------------------------------------
# random inputs for the pins
# ---------------------------------------------------------------------------
def rand_ad(R, C, S, gen, p=0.3, wmax=None):
    """Random anti-distance matrix: each entry present with probability p,
    with distance uniform in [0, wmax] (wmax defaults to S, so some entries
    are at or beyond saturation)."""
    wmax = S if wmax is None else wmax
    present = gen.random((R, C)) < p
    w = gen.integers(0, wmax + 1, size=(R, C))
    return np.where(present & (w < S), S - w, 0).astype(np.int64)


def rand_bool(R, C, gen, p=0.3):
    return (gen.random((R, C)) < p).astype(np.uint8)


def identity(D, one):
    return (np.eye(D, dtype=np.int64) * one)


# ---------------------------------------------------------------------------
# pins on a product implementation mul(A, B, S) -> int array
# ---------------------------------------------------------------------------
def pin_ad_mul_scalar_table(mul, S, a_values=None):
    """Exhaustive (or dense) scalar table through 1-column by 1-row products:
    C = a (column) * b (row) has C_ij = a_i (x) b_j.  Compared with the
    Sec. IV listing form (b > S - a ? b - (S - a) : 0) and the De Morgan form
    S - min((S - a) + (S - b), S)."""
    a = np.arange(S + 1, dtype=np.int64) if a_values is None else np.asarray(a_values, np.int64)
    b = np.arange(S + 1, dtype=np.int64)
    C = np.asarray(mul(a[:, None], b[None, :], S), np.int64)
    na = (S - a)[:, None]
    listing = np.where(b[None, :] > na, b[None, :] - na, 0)
    demorgan = S - np.minimum((S - a)[:, None] + (S - b)[None, :], S)
    assert np.array_equal(C, listing), "scalar table differs from the listing form"
    assert np.array_equal(C, demorgan), "scalar table differs from the De Morgan form"


def pin_ad_mul_random(mul, S, gen, shapes=((1, 1, 1), (3, 5, 2), (17, 9, 23), (40, 33, 31),
                                             (16, 16, 16))):
    for (R, K, N) in shapes:
        A = rand_ad(R, K, S, gen)
        B = rand_ad(K, N, S, gen)
        C = np.asarray(mul(A, B, S), np.int64)
        assert np.array_equal(C, ad_product_demorgan(A, B, S)), "product != De Morgan dual"
        assert np.array_equal(C, ad_product_shortest_path(A, B, S)), \
            "product != layered shortest path"


def pin_ad_mul_boolean_reduction(mul, S, gen, R=19, K=23, N=17):
    """Entries restricted to {0, S}: anti-distance product = S x Boolean
    product of the supports (Sec. III: 1 = distance 0, 0 = infinity)."""
    Ab = rand_bool(R, K, gen)
    Bb = rand_bool(K, N, gen)
    C = np.asarray(mul(Ab.astype(np.int64) * S, Bb.astype(np.int64) * S, S), np.int64)
    assert np.array_equal(C, bool_product_matmul(Ab, Bb).astype(np.int64) * S)


def pin_ad_mul_laws(mul, S, gen, D=13):
    A, B, C = (rand_ad(D, D, S, gen, p=0.5) for _ in range(3))
    I = identity(D, S)
    m = lambda X, Y: np.asarray(mul(X, Y, S), np.int64)
    assert np.array_equal(m(I, A), A) and np.array_equal(m(A, I), A), "identity law"
    assert np.array_equal(m(m(A, B), C), m(A, m(B, C))), "associativity"
    assert np.array_equal(m(A, np.maximum(B, C)), np.maximum(m(A, B), m(A, C))), \
        "left distributivity"
    assert np.array_equal(m(np.maximum(A, B), C), np.maximum(m(A, C), m(B, C))), \
        "right distributivity"
    Z = np.zeros((D, D), np.int64)
    assert not m(Z, A).any() and not m(A, Z).any(), "zero annihilates"


def pin_bool_mul(mul, gen):
    """Exhaustive 3 x 3 Boolean products (all 2^9 x 2^9 pairs), then random
    rectangular shapes, against integer matmul."""
    allm = ((np.arange(512)[:, None] >> np.arange(9)[None, :]) & 1).astype(np.uint8)
    mats = allm.reshape(512, 3, 3)
    Astack = mats.reshape(512 * 3, 3)
    Bstack = np.concatenate(list(mats), axis=1)
    C = np.asarray(mul(Astack, Bstack), np.int64)
    assert np.array_equal(C, bool_product_matmul(Astack, Bstack)), "3x3 exhaustive"
    for (R, K, N) in ((1, 1, 1), (7, 65, 130), (64, 64, 64), (33, 129, 70)):
        A = rand_bool(R, K, gen)
        B = rand_bool(K, N, gen)
        assert np.array_equal(np.asarray(mul(A, B), np.int64), bool_product_matmul(A, B))


# ---------------------------------------------------------------------------
# pins on a closure implementation clo(A, S) -> int array
# ---------------------------------------------------------------------------
def closed_form_cycle(D, S, w=1):
    """Directed D-cycle i -> i+1 (mod D), every edge of distance w: the
    distance from i to j over >= 1 edge is w * (((j - i - 1) mod D) + 1)."""
    i = np.arange(D)[:, None]
    j = np.arange(D)[None, :]
    d = w * (((j - i - 1) % D) + 1)
    return np.where(d >= S, 0, S - np.minimum(d, S))


def cycle_matrix(D, S, w=1):
    A = np.zeros((D, D), np.int64)
    if D:
        A[np.arange(D), (np.arange(D) + 1) % D] = max(S - w, 0)
    return A


def pin_ad_closure_closed_forms(clo, S):
    for D, w in ((1, 1), (2, 3), (5, 1), (40, 1), (70, 4), (300, 1)):
        assert np.array_equal(np.asarray(clo(cycle_matrix(D, S, w), S), np.int64),
                              closed_form_cycle(D, S, w)), "cycle D=%d w=%d" % (D, w)
    for D in (1, 4, 9):
        full = np.full((D, D), S, np.int64)
        assert np.array_equal(np.asarray(clo(full, S), np.int64), full), "all-S complete graph"
    Z = np.zeros((6, 6), np.int64)
    assert not np.asarray(clo(Z, S)).any(), "empty graph"
    # a single self loop of distance w gives exactly that diagonal entry
    A = np.zeros((3, 3), np.int64)
    A[1, 1] = S - 7
    T = np.asarray(clo(A, S), np.int64)
    assert T[1, 1] == S - 7 and T.sum() == S - 7, "self loop"


def pin_ad_closure_bruteforce(clo, S, gen, sizes=(1, 2, 3, 6, 11, 17, 24), trials=3):
    for D in sizes:
        for _ in range(trials):
            wmax = S if gen.random() < 0.5 else max(1, S // 4)
            A = rand_ad(D, D, S, gen, p=float(gen.uniform(0.05, 0.5)), wmax=wmax)
            T = np.asarray(clo(A, S), np.int64)
            assert np.array_equal(T, ad_closure_bellman_ford(A, S)), "Bellman-Ford D=%d" % D


def pin_ad_closure_networkx(clo, S, gen, sizes=(40, 97)):
    for D in sizes:
        A = rand_ad(D, D, S, gen, p=0.06, wmax=S // 3)
        T = np.asarray(clo(A, S), np.int64)
        assert np.array_equal(T, ad_closure_networkx(A, S)), "networkx D=%d" % D


def pin_ad_closure_invariants(clo, mul, S, gen, D=29):
    A = rand_ad(D, D, S, gen, p=0.12, wmax=S // 3)
    T = np.asarray(clo(A, S), np.int64)
    m = lambda X, Y: np.asarray(mul(X, Y, S), np.int64)
    assert np.array_equal(np.maximum(T, m(T, T)), T), "idempotence T (+) T*T = T"
    assert np.array_equal(np.maximum(A, m(A, T)), T), "fixed point T = A (+) A*T"
    assert np.array_equal(np.maximum(A, m(T, A)), T), "fixed point T = A (+) T*A"
    assert np.array_equal(np.asarray(clo(T, S), np.int64), T), "closure of a closure"
    assert (T >= A).all(), "T >= A"
    assert np.array_equal(np.asarray(clo(A.T.copy(), S), np.int64), T.T), "transpose"
    perm = gen.permutation(D)
    P = A[np.ix_(perm, perm)]
    assert np.array_equal(np.asarray(clo(P, S), np.int64), T[np.ix_(perm, perm)]), "permutation"
    E = np.zeros((D + 5, D + 5), np.int64)
    E[:D, :D] = A
    TE = np.asarray(clo(E, S), np.int64)
    assert np.array_equal(TE[:D, :D], T) and not TE[D:].any() and not TE[:, D:].any(), \
        "zero padding"


def pin_product_equals_warshall(clo, mul, S, gen, D=21):
    """Sec. II: A (+) A*A (+) ... = A * (I (+) A)^(D'-1) for every D' >= D,
    with the power taken by repeated squaring of (I (+) A)."""
    A = rand_ad(D, D, S, gen, p=0.15, wmax=S // 2)
    m = lambda X, Y: np.asarray(mul(X, Y, S), np.int64)
    P = np.maximum(identity(D, S), A)
    for _ in range(int(math.ceil(math.log2(max(D - 1, 2))))):
        P = m(P, P)
    assert np.array_equal(m(A, P), np.asarray(clo(A, S), np.int64)), "A*(I+A)^(D'-1)"


def pin_bool_closure(clo, gen, sizes=(1, 2, 5, 16, 37, 64)):
    for D in sizes:
        for p in (0.03, 0.1, 0.3):
            A = rand_bool(D, D, gen, p)
            T = np.asarray(clo(A), np.int64)
            assert np.array_equal(T, bool_closure_bfs(A)), "BFS D=%d" % D
            assert np.array_equal(T, bool_closure_networkx(A)), "networkx D=%d" % D
    A = np.zeros((9, 9), np.uint8)
    A[np.arange(9), (np.arange(9) + 1) % 9] = 1
    assert np.array_equal(np.asarray(clo(A), np.int64), np.ones((9, 9))), "cycle"
    A[8, 0] = 0  # a path 0 -> 1 -> ... -> 8: strictly upper triangle
    assert np.array_equal(np.asarray(clo(A), np.int64), np.triu(np.ones((9, 9)), 1)), "path"


def golden_read(path):
    """Parse a golden file: key/value lines and named integer matrices."""
    out = {}
    cur = None
    with open(path) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            tok = line.split()
            if len(tok) == 1 and tok[0].isalpha():
                cur = tok[0]
                out[cur] = []
            elif len(tok) == 2 and tok[0].isalpha():
                out[tok[0]] = int(tok[1])
                cur = None
            else:
                out.setdefault(cur, []).append([int(t) for t in tok])
    return {k: (np.array(v, np.int64) if isinstance(v, list) else v) for k, v in out.items()}


def golden_rows(path):
    rows = []
    with open(path) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                rows.append(line.split())
    return rows


__all__ = [n for n in dir() if n.startswith(("pin_", "bool_", "ad_", "closed_", "cycle_",
                                             "rand_", "golden_"))] + ["identity", "synthgen"]
