"""The oracle against independent pins (no GPU).

Every oracle function is checked here against something that shares no code
with it: hand-derived golden values, closed forms, brute force, library
routines (integer matmul, scipy and networkx shortest paths / reachability)
and the algebraic laws the paper states.
"""
import os

import numpy as np
import pytest

import oracle
import synthgen
from pins import (
    ad_closure_bellman_ford, bool_closure_bfs, golden_read, golden_rows,
    pin_ad_closure_bruteforce, pin_ad_closure_closed_forms, pin_ad_closure_invariants,
    pin_ad_closure_networkx, pin_ad_mul_boolean_reduction, pin_ad_mul_laws,
    pin_ad_mul_random, pin_ad_mul_scalar_table, pin_bool_closure, pin_bool_mul,
    pin_product_equals_warshall, rand_ad, rand_bool,
)

SCALES = (255, 65535, 2 ** 32 - 1)


def o_mul(A, B, S):
    return oracle.ad_mul(A, B, S)


def o_clo(A, S):
    return oracle.ad_closure(A, S)


def o_clo_rows(A, S):
    A = np.asarray(A)
    return oracle.ad_closure_rows(A, S, np.arange(A.shape[0]))


def o_bool_mul(A, B):
    return oracle.bool_mul(A, B)


def o_bool_mul_words(A, B):
    A = np.asarray(A, np.uint8)
    B = np.asarray(B, np.uint8)
    K, N = B.shape
    Aw = synthgen.pack_bits(A, synthgen.aligned_ld_words(A.shape[1]))
    Bw = synthgen.pack_bits(B, synthgen.aligned_ld_words(N))
    return synthgen.unpack_bits(oracle.bool_mul_words(Aw, Bw, K, N), N)


def o_bool_clo(A):
    return oracle.bool_closure(A)


def o_bool_clo_words(A):
    A = np.asarray(A, np.uint8)
    D = A.shape[0]
    T = oracle.bool_closure_words(synthgen.pack_bits(A, synthgen.aligned_ld_words(D)), D)
    return synthgen.unpack_bits(T, D)


def o_bool_clo_rows(A):
    A = np.asarray(A, np.uint8)
    D = A.shape[0]
    rows = oracle.bool_closure_rows_words(synthgen.pack_bits(A), D, np.arange(D))
    return synthgen.unpack_bits(rows, D)


# ---------------------------------------------------------------------------
# golden, hand-derived values
# ---------------------------------------------------------------------------
def test_golden_scales(golden_dir):
    rows = golden_rows(os.path.join(golden_dir, "tab1_scales.txt"))
    table = {r[0]: int(r[1]) for r in rows}
    assert oracle.scale(np.uint8) == table["uint8"] == oracle.S_U8
    assert oracle.scale(np.uint16) == table["uint16"] == oracle.S_U16
    assert table["uint32"] == 2 ** 32 - 1


@pytest.mark.parametrize("name", ["worked_closure_u8.txt", "worked_closure_u16.txt"])
def test_golden_worked_closure(golden_dir, name):
    g = golden_read(os.path.join(golden_dir, name))
    S, A = g["S"], g["A"]
    assert np.array_equal(oracle.ad_mul(A, A, S), g["AA"])
    assert np.array_equal(oracle.ad_closure(A, S), g["CLOSURE"])
    assert np.array_equal(oracle.ad_closure_rows(A, S, np.arange(g["D"])), g["CLOSURE"])


def test_golden_saturation(golden_dir):
    for S, w1, w2, expect in golden_rows(os.path.join(golden_dir, "worked_saturation.txt")):
        S, w1, w2, expect = int(S), int(w1), int(w2), int(expect)
        A = np.zeros((3, 3), np.int64)
        A[0, 1] = S - w1
        A[1, 2] = S - w2
        assert oracle.ad_mul(A, A, S)[0, 2] == expect
        assert oracle.ad_closure(A, S)[0, 2] == expect
        assert oracle.ad_closure_rows(A, S, [0])[0, 2] == expect


def test_golden_bool(golden_dir):
    g = golden_read(os.path.join(golden_dir, "worked_bool.txt"))
    A = g["A"]
    assert np.array_equal(oracle.bool_mul(A, A), g["AA"])
    assert np.array_equal(oracle.bool_closure(A), g["CLOSURE"])
    assert np.array_equal(o_bool_clo_words(A), g["CLOSURE"])
    assert np.array_equal(o_bool_clo_rows(A), g["CLOSURE"])
    assert np.array_equal(o_bool_mul_words(A, A), g["AA"])


# ---------------------------------------------------------------------------
# products
# ---------------------------------------------------------------------------
def test_scalar_table_u8_exhaustive():
    pin_ad_mul_scalar_table(o_mul, 255)


def test_scalar_table_u16_dense():
    gen = synthgen.generator(11)
    a = np.unique(np.concatenate([
        [0, 1, 2, 3, 254, 255, 256, 32767, 32768, 65533, 65534, 65535],
        gen.integers(0, 65536, size=180)]))
    pin_ad_mul_scalar_table(o_mul, 65535, a_values=a)


def test_scalar_table_u32_sampled():
    """S = 2^32 - 1 (uint32 entries): the scalar table on sampled operands,
    extremes and the int32 boundary included, against the listing and De
    Morgan forms (the int64 loops of the oracle)."""
    S = 2 ** 32 - 1
    gen = synthgen.generator(19)
    special = [0, 1, 2, 2 ** 31 - 1, 2 ** 31, 2 ** 31 + 1, S - 2, S - 1, S]
    a = np.unique(np.concatenate([special, gen.integers(0, S + 1, size=120)])).astype(np.int64)
    b = np.unique(np.concatenate([special, gen.integers(0, S + 1, size=120)])).astype(np.int64)
    C = np.asarray(o_mul(a[:, None], b[None, :], S), np.int64)
    na = (S - a)[:, None]
    assert np.array_equal(C, np.where(b[None, :] > na, b[None, :] - na, 0))
    assert np.array_equal(C, S - np.minimum((S - a)[:, None] + (S - b)[None, :], S))


@pytest.mark.parametrize("S", SCALES)
def test_ad_mul_random(S):
    pin_ad_mul_random(o_mul, S, synthgen.generator(12 + S))


@pytest.mark.parametrize("S", SCALES)
def test_ad_mul_boolean_reduction(S):
    pin_ad_mul_boolean_reduction(o_mul, S, synthgen.generator(13))


@pytest.mark.parametrize("S", SCALES)
def test_ad_mul_laws(S):
    pin_ad_mul_laws(o_mul, S, synthgen.generator(14))


def test_ad_mul_accumulate():
    gen = synthgen.generator(15)
    for S in SCALES:
        A, B, C = rand_ad(9, 11, S, gen), rand_ad(11, 7, S, gen), rand_ad(9, 7, S, gen)
        assert np.array_equal(oracle.ad_mul(A, B, S, C=C), np.maximum(C, oracle.ad_mul(A, B, S)))


def test_ad_mul_empty_inner():
    A = np.zeros((3, 0), np.int64)
    B = np.zeros((0, 4), np.int64)
    assert not oracle.ad_mul(A, B, 255).any()
    C = np.full((3, 4), 9)
    assert (oracle.ad_mul(A, B, 255, C=C) == 9).all()


def test_bool_mul_bytes():
    pin_bool_mul(o_bool_mul, synthgen.generator(16))


def test_bool_mul_words():
    pin_bool_mul(o_bool_mul_words, synthgen.generator(17))


def test_bool_mul_words_accumulate_and_padding():
    gen = synthgen.generator(18)
    A, B, C = rand_bool(13, 70, gen), rand_bool(70, 100, gen), rand_bool(13, 100, gen)
    ldw = synthgen.aligned_ld_words(100)
    got = oracle.bool_mul_words(synthgen.pack_bits(A, 2), synthgen.pack_bits(B, ldw), 70, 100,
                                C=synthgen.pack_bits(C, ldw))
    assert synthgen.padding_bits_clear(got, 100)
    want = np.maximum(C, (A.astype(int) @ B.astype(int) > 0).astype(np.uint8))
    assert np.array_equal(synthgen.unpack_bits(got, 100), want)


# ---------------------------------------------------------------------------
# closures
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("S", SCALES)
@pytest.mark.parametrize("impl", ["warshall", "rows"])
def test_ad_closure_closed_forms(S, impl):
    pin_ad_closure_closed_forms(o_clo if impl == "warshall" else o_clo_rows, S)


@pytest.mark.parametrize("S", SCALES)
@pytest.mark.parametrize("impl", ["warshall", "rows"])
def test_ad_closure_bruteforce(S, impl):
    pin_ad_closure_bruteforce(o_clo if impl == "warshall" else o_clo_rows, S,
                              synthgen.generator(20 + S))


@pytest.mark.parametrize("S", SCALES)
def test_ad_closure_networkx(S):
    pin_ad_closure_networkx(o_clo, S, synthgen.generator(21))
    pin_ad_closure_networkx(o_clo_rows, S, synthgen.generator(22))


@pytest.mark.parametrize("S", SCALES)
def test_ad_closure_invariants(S):
    pin_ad_closure_invariants(o_clo, o_mul, S, synthgen.generator(23))


@pytest.mark.parametrize("S", SCALES)
def test_product_equals_warshall(S):
    pin_product_equals_warshall(o_clo, o_mul, S, synthgen.generator(24))


def test_ad_closure_aliased_mul_loop():
    """Sec. III: running the multiplication loop with P, A and B all the same
    in-place matrix T is Warshall's algorithm.  The oracle's Warshall steps
    one k at a time; taking one step with T as both operands of a one-column
    by one-row product reproduces it step by step."""
    gen = synthgen.generator(25)
    S = 255
    A = rand_ad(15, 15, S, gen, p=0.2)
    T = A.copy()
    for k in range(15):
        T = oracle.ad_mul(T[:, k:k + 1], T[k:k + 1, :], S, C=T)
        assert np.array_equal(T, oracle.ad_closure(A, S, k_end=k + 1))
    assert np.array_equal(T, oracle.ad_closure(A, S))


def test_ad_closure_u8_two_hop_saturation():
    """uint8 with distances in [1, 200]: paths of total distance >= 255 read
    as absent; compare with the brute force on a configuration-4 style graph."""
    gen = synthgen.generator(26)
    rows, cols = synthgen.bernoulli_edges(23, 0.2, gen)
    w = gen.integers(1, 201, size=len(rows))
    A = synthgen.encode_antidist(23, rows, cols, w, np.uint8).astype(np.int64)
    assert np.array_equal(oracle.ad_closure(A, 255), ad_closure_bellman_ford(A, 255))


@pytest.mark.parametrize("impl", ["bytes", "words", "rows"])
def test_bool_closure(impl):
    fn = {"bytes": o_bool_clo, "words": o_bool_clo_words, "rows": o_bool_clo_rows}[impl]
    pin_bool_closure(fn, synthgen.generator(27))


def test_bool_closure_matches_antidist_reduction():
    """Boolean closure = anti-distance closure of the {0, S} matrix / S."""
    gen = synthgen.generator(28)
    A = rand_bool(31, 31, gen, 0.06)
    assert np.array_equal(oracle.bool_closure(A).astype(np.int64) * 255,
                          oracle.ad_closure(A.astype(np.int64) * 255, 255))


def test_closure_rows_agree_with_warshall_medium():
    gen = synthgen.generator(29)
    A = synthgen.cfg_antidist(D=200, seed=77)[:, :200].astype(np.int64)
    rows = np.sort(gen.choice(200, size=12, replace=False))
    assert np.array_equal(oracle.ad_closure_rows(A, 65535, rows),
                          oracle.ad_closure(A, 65535)[rows])
    Ab = synthgen.unpack_bits(synthgen.cfg_bool16384(D=300, seed=5, planted_blocks=2, block=40),
                              300)
    T = oracle.bool_closure(Ab)
    assert np.array_equal(o_bool_clo_rows(Ab), T)
    assert np.array_equal(T, bool_closure_bfs(Ab))


def test_openmp_threads_do_not_change_results():
    A = synthgen.cfg_antidist(D=160, seed=3)[:, :160]
    oracle.set_threads(1)
    T1 = oracle.ad_closure(A, 65535)
    oracle.set_threads(4)
    T4 = oracle.ad_closure(A, 65535)
    oracle.set_threads(1)
    assert np.array_equal(T1, T4)
