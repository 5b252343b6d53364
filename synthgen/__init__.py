"""Seeded synthetic graph inputs, shared by the tests, the benchmark and the
smoke check.

This module holds none of the semiring arithmetic: it only draws random
digraphs and edge weights, writes them into the storage formats the library
and the oracle both take, and packs / unpacks Boolean bit rows.

Storage formats
---------------
* Anti-distance matrices (Sec. III, scaled to integers as in Sec. IV): entry
  (i, j) of an edge i -> j with distance w is S - w; an absent edge is 0 (the
  additive zero, "distance infinity"); a distance of 0 gives S (the
  multiplicative one); distances w >= S cannot be told from absent edges and
  are stored as 0.  S = 255 for uint8 and 65535 for uint16.  Row-major with a
  leading dimension ``ld`` >= D (in elements); padding columns are zero.
* Boolean matrices (Sec. II): entry (i, j) = 1 for an edge i -> j (row =
  source, as in the index formula of the product).  Bit-packed in uint64 words,
  entry (r, c) at bit c % 64 of word c // 64 of row r (least significant bit
  first, the byte/bit order of the paper's Boolean listing in Sec. IV);
  padding bits are zero.

Random digraphs are i.i.d. Bernoulli(p) over ordered pairs i != j (no self
loops), drawn row block by row block from ``numpy.random.Generator(PCG64)``.
"""
import math

import numpy as np

SEED_BASE = 170508743

S_BY_DTYPE = {np.dtype(np.uint8): 255, np.dtype(np.uint16): 65535,
              np.dtype(np.uint32): 2 ** 32 - 1}


def generator(seed):
    return np.random.Generator(np.random.PCG64(seed))


def config_seed(config_index: int) -> int:
    """Seed of workload configuration ``config_index`` (1-based)."""
    return SEED_BASE + int(config_index)


def round_up(x: int, m: int) -> int:
    return (x + m - 1) // m * m


def aligned_ld(ncols: int, dtype) -> int:
    """Smallest leading dimension >= ncols whose rows are 16-byte multiples."""
    per16 = 16 // np.dtype(dtype).itemsize
    return max(per16, round_up(ncols, per16))


def aligned_ld_words(ncols: int) -> int:
    """Words per packed Boolean row, rounded to an even count (16 bytes)."""
    return max(2, round_up((ncols + 63) // 64, 2))


# ---------------------------------------------------------------------------
# random digraphs
# ---------------------------------------------------------------------------
def bernoulli_edges(D: int, p: float, gen, chunk_rows: int = 1024):
    """Edges (rows, cols) of a digraph with each ordered pair i != j present
    independently with probability p.  Rows are in ascending order."""
    rows, cols = [], []
    for r0 in range(0, D, chunk_rows):
        r1 = min(D, r0 + chunk_rows)
        mask = gen.random((r1 - r0, D)) < p
        idx = np.arange(r0, r1)
        mask[idx - r0, idx] = False
        rr, cc = np.nonzero(mask)
        rows.append(rr.astype(np.int64) + r0)
        cols.append(cc.astype(np.int64))
    if not rows:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    return np.concatenate(rows), np.concatenate(cols)


def antidist_weights(n_edges: int, wlo: int, whi: int, gen, heavy_frac: float = 0.0,
                     heavy_lo: int = 64536, heavy_hi: int = 65534):
    """Edge distances uniform in [wlo, whi]; a fraction ``heavy_frac`` of the
    edges instead draws from [heavy_lo, heavy_hi] (distances near 65535)."""
    w = gen.integers(wlo, whi + 1, size=n_edges, dtype=np.int64)
    if heavy_frac > 0:
        heavy = gen.random(n_edges) < heavy_frac
        w[heavy] = gen.integers(heavy_lo, heavy_hi + 1, size=int(heavy.sum()), dtype=np.int64)
    return w


def encode_antidist(D: int, rows, cols, weights, dtype, ld: int = None, ncols: int = None):
    """Anti-distance matrix with entry S - w at each edge (0 where w >= S)."""
    dtype = np.dtype(dtype)
    S = S_BY_DTYPE[dtype]
    ncols = D if ncols is None else ncols
    ld = ncols if ld is None else ld
    if ld < ncols:
        raise ValueError("ld < number of columns")
    M = np.zeros((D, ld), dtype)
    w = np.asarray(weights, np.int64)
    keep = w < S
    M[np.asarray(rows)[keep], np.asarray(cols)[keep]] = (S - w[keep]).astype(dtype)
    return M


def antidist_graph(D: int, p: float, wlo: int, whi: int, dtype, gen, heavy_frac: float = 0.0,
                   ld: int = None):
    rows, cols = bernoulli_edges(D, p, gen)
    w = antidist_weights(len(rows), wlo, whi, gen, heavy_frac)
    return encode_antidist(D, rows, cols, w, dtype, ld)


def bool_dense(D: int, rows, cols, ncols: int = None):
    ncols = D if ncols is None else ncols
    M = np.zeros((D, ncols), np.uint8)
    M[np.asarray(rows), np.asarray(cols)] = 1
    return M


def planted_cycles(D: int, n_blocks: int, block: int, gen):
    """Edges of ``n_blocks`` disjoint directed cycles, each through ``block``
    randomly chosen vertices in random order (each block strongly connected)."""
    if n_blocks * block > D:
        raise ValueError("blocks do not fit")
    perm = gen.permutation(D)[: n_blocks * block].reshape(n_blocks, block)
    src = perm.reshape(-1)
    dst = np.roll(perm, -1, axis=1).reshape(-1)
    return src.astype(np.int64), dst.astype(np.int64)


# ---------------------------------------------------------------------------
# Boolean bit packing
# ---------------------------------------------------------------------------
def pack_bits(dense01, ld_words: int = None):
    """uint8 {0,1} R x C -> uint64 R x ld_words, LSB-first, zero padding."""
    dense01 = np.ascontiguousarray(dense01, dtype=np.uint8)
    R, C = dense01.shape
    nw = (C + 63) // 64
    ld_words = nw if ld_words is None else ld_words
    if ld_words < nw:
        raise ValueError("ld_words too small")
    padded = np.zeros((R, ld_words * 64), np.uint8)
    padded[:, :C] = dense01
    by = np.packbits(padded, axis=1, bitorder="little")
    return np.ascontiguousarray(by).view("<u8").reshape(R, ld_words).astype(np.uint64)


def unpack_bits(words, ncols: int):
    """uint64 R x W words -> uint8 {0,1} R x ncols."""
    words = np.ascontiguousarray(words, dtype=np.uint64)
    R = words.shape[0]
    by = words.astype("<u8").view(np.uint8).reshape(R, -1)
    bits = np.unpackbits(by, axis=1, bitorder="little")
    return np.ascontiguousarray(bits[:, :ncols])


def padding_bits_clear(words, ncols: int) -> bool:
    """True when every bit at column >= ncols of every row is zero."""
    words = np.ascontiguousarray(words, dtype=np.uint64)
    full = unpack_bits(words, words.shape[1] * 64)
    return not full[:, ncols:].any()


def bool_graph_packed(D: int, p: float, gen, planted_blocks: int = 0, block: int = 0,
                      ld_words: int = None):
    rows, cols = bernoulli_edges(D, p, gen)
    if planted_blocks:
        pr, pc = planted_cycles(D, planted_blocks, block, gen)
        rows = np.concatenate([rows, pr])
        cols = np.concatenate([cols, pc])
    return pack_bits(bool_dense(D, rows, cols), ld_words)


# ---------------------------------------------------------------------------
# the five workload configurations
# ---------------------------------------------------------------------------
def cfg_bool256(seed: int = None):
    """Boolean 256 x 256 random digraph, p = 0.02 (packed, 4 words per row)."""
    gen = generator(config_seed(1) if seed is None else seed)
    return bool_graph_packed(256, 0.02, gen, ld_words=aligned_ld_words(256))


def cfg_antidist(D: int = 1024, seed: int = None, dtype=np.uint16, which: int = 0):
    """Anti-distance random digraph, p = 0.05, distances uniform in [1, 1000],
    1% of the edges with distances in [64536, 65534] (uint16).  ``which``
    selects independent matrices (A = 0, B = 1) of the same configuration.
    For uint8 the heavy edges and distances >= 255 read as absent."""
    base = config_seed(2) if seed is None else seed
    ss = np.random.SeedSequence(base).spawn(which + 1)[which]
    gen = np.random.Generator(np.random.PCG64(ss))
    return antidist_graph(D, 0.05, 1, 1000, dtype, gen, heavy_frac=0.01, ld=aligned_ld(D, dtype))


def cfg_antidist_u8(D: int = 8192, seed: int = None):
    """uint8 variant: p = 0.05, distances uniform in [1, 200]."""
    gen = generator(config_seed(2) + 100 if seed is None else seed)
    return antidist_graph(D, 0.05, 1, 200, np.uint8, gen, ld=aligned_ld(D, np.uint8))


def cfg_bool16384(D: int = 16384, seed: int = None, planted_blocks: int = 8, block: int = 512):
    """Boolean closure input: mean out-degree 3 plus planted strongly connected
    blocks (directed cycles through random vertex sets)."""
    gen = generator(config_seed(3) if seed is None else seed)
    p = 3.0 / (D - 1)
    nb = planted_blocks if planted_blocks * block <= D else 0
    return bool_graph_packed(D, p, gen, nb, block, ld_words=aligned_ld_words(D))


def batch_sizes(count: int, nlo: int, nhi: int, gen):
    """Vertex counts log-uniform in [nlo, nhi], rounded to integers."""
    u = gen.uniform(math.log(nlo), math.log(nhi), size=count)
    return np.clip(np.rint(np.exp(u)).astype(np.int64), nlo, nhi)


def cfg_batch(count: int = 4096, nlo: int = 32, nhi: int = 1024, seed: int = None):
    """Batched workload: ``count`` digraphs with log-uniform vertex counts,
    density uniform in [0.01, 0.2] and distances uniform in [1, 200].
    Returns a list of (n, rows, cols, weights); encode with
    ``encode_antidist`` for uint8 or uint16 (same topology and distances)."""
    gen = generator(config_seed(4) if seed is None else seed)
    ns = batch_sizes(count, nlo, nhi, gen)
    ps = gen.uniform(0.01, 0.2, size=count)
    out = []
    for n, p in zip(ns, ps):
        rows, cols = bernoulli_edges(int(n), float(p), gen)
        w = gen.integers(1, 201, size=len(rows), dtype=np.int64)
        out.append((int(n), rows, cols, w))
    return out


def serving_trace(count: int, nlo: int = 64, nhi: int = 8192, seed: int = None):
    """Request trace: (n, kind) pairs with n log-uniform in [nlo, nhi] and
    kind 'bool' or 'u16' with probability 1/2 each, plus per-request seeds.
    Arrival times are drawn separately once the service rate is known."""
    gen = generator(config_seed(5) if seed is None else seed)
    ns = batch_sizes(count, nlo, nhi, gen)
    kinds = np.where(gen.random(count) < 0.5, "bool", "u16")
    seeds = gen.integers(0, 2 ** 62, size=count)
    return [(int(n), str(k), int(s)) for n, k, s in zip(ns, kinds, seeds)]


def serving_request(n: int, kind: str, seed: int):
    """Input matrix of one serving request: Boolean as the 256-vertex
    workload (p = 0.02) or uint16 anti-distance as the 1024-vertex one
    (p = 0.05)."""
    gen = generator(seed)
    if kind == "bool":
        return bool_graph_packed(n, 0.02, gen, ld_words=aligned_ld_words(n))
    return antidist_graph(n, 0.05, 1, 1000, np.uint16, gen, heavy_frac=0.01,
                          ld=aligned_ld(n, np.uint16))


def poisson_arrivals(count: int, rate: float, gen):
    """Arrival times (seconds from 0) of a Poisson process of the given rate."""
    return np.cumsum(gen.exponential(1.0 / rate, size=count))
