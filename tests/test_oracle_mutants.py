"""Planted mistakes in copies of the oracle's loops must fail the pins.

Each mutant below is the oracle's algorithm with one plausible mistake (a
dropped term, an off-by-one in the saturation, a transposed operand, a wrong
index, a wrong starting value).  The pins of ``pins.py`` are run on each
mutant and at least one must fail; the unmutated copy must pass them all.
Everything runs on the CPU.
"""
import numpy as np
import pytest

import synthgen
from pins import (
    pin_ad_closure_bruteforce, pin_ad_closure_closed_forms, pin_ad_closure_invariants,
    pin_ad_closure_networkx, pin_ad_mul_boolean_reduction, pin_ad_mul_laws,
    pin_ad_mul_random, pin_ad_mul_scalar_table, pin_bool_closure, pin_bool_mul,
    pin_product_equals_warshall,
)


# ---- products: P := 0; for k: P := P (+) A[:, k] * B[k, :] -----------------
def mul_ok(A, B, S, otimes=None, klimit=None, swap=False, init=0):
    A = np.asarray(A, np.int64)
    B = np.asarray(B, np.int64)
    if swap:
        A, B = B.T, A.T
    otimes = otimes or (lambda a, b: np.maximum(a + b - S, 0))
    R, K = A.shape
    P = np.full((R, B.shape[1]), init, np.int64)
    for k in range(K if klimit is None else min(K, klimit(K))):
        P = np.maximum(P, otimes(A[:, k:k + 1], B[k:k + 1, :]))
    return P.T if swap else P


MUL_MUTANTS = {
    "offbyone": lambda A, B, S: mul_ok(A, B, S, otimes=lambda a, b: np.maximum(a + b - S + 1, 0)),
    "wraparound": lambda A, B, S: mul_ok(A, B, S, otimes=lambda a, b: (a + b - S) % (S + 1)),
    "minplus_plain": lambda A, B, S: mul_ok(A, B, S, otimes=lambda a, b: np.minimum(a, b)),
    "drop_last_k": lambda A, B, S: mul_ok(A, B, S, klimit=lambda K: K - 1),
    "b_transposed": lambda A, B, S: mul_ok(A, np.asarray(B).T if np.asarray(B).shape[0] ==
                                           np.asarray(B).shape[1] else B, S),
    "swapped": lambda A, B, S: mul_ok(B, A, S) if np.asarray(A).shape == np.asarray(B).shape
    else mul_ok(A, B, S),
    "init_one": lambda A, B, S: mul_ok(A, B, S, init=1),
}


def run_mul_pins(mul):
    pin_ad_mul_scalar_table(mul, 255)
    for S in (255, 65535):
        pin_ad_mul_random(mul, S, synthgen.generator(101))
        pin_ad_mul_boolean_reduction(mul, S, synthgen.generator(102))
        pin_ad_mul_laws(mul, S, synthgen.generator(103))


def test_mul_copy_passes():
    run_mul_pins(mul_ok)


@pytest.mark.parametrize("name", sorted(MUL_MUTANTS))
def test_mul_mutant_caught(name):
    with pytest.raises(AssertionError):
        run_mul_pins(MUL_MUTANTS[name])


# ---- closures: T := A; for k: T := T (+) T[:, k] * T[k, :] -----------------
def clo_ok(A, S, variant=None):
    T = np.asarray(A, np.int64).copy()
    D = T.shape[0]
    ot = lambda a, b: np.maximum(a + b - S, 0)
    if variant == "reflexive_start":
        T = np.maximum(T, np.eye(D, dtype=np.int64) * S)
    if variant == "ijk_order":
        # the product loop order used as if it were a closure: one pass over
        # (i, j) with k innermost is not Warshall's algorithm
        for i in range(D):
            for j in range(D):
                for k in range(D):
                    T[i, j] = max(T[i, j], ot(T[i, k], T[k, j]))
        return T
    for k in range(D if variant != "skip_last" else max(D - 1, 0)):
        if variant == "wrong_index":
            col = T[k, :].reshape(-1, 1)
        else:
            col = T[:, k:k + 1]
        T = np.maximum(T, ot(col, T[k:k + 1, :]))
    return T


CLO_MUTANTS = {
    "reflexive_start": lambda A, S: clo_ok(A, S, "reflexive_start"),
    "ijk_order": lambda A, S: clo_ok(A, S, "ijk_order"),
    "skip_last": lambda A, S: clo_ok(A, S, "skip_last"),
    "wrong_index": lambda A, S: clo_ok(A, S, "wrong_index"),
    "one_product": lambda A, S: np.maximum(np.asarray(A, np.int64), mul_ok(A, A, S)),
}


def run_clo_pins(clo):
    for S in (255, 65535):
        pin_ad_closure_closed_forms(clo, S)
        pin_ad_closure_bruteforce(clo, S, synthgen.generator(104), sizes=(3, 6, 11), trials=3)
        pin_ad_closure_networkx(clo, S, synthgen.generator(105), sizes=(30,))
        pin_ad_closure_invariants(clo, mul_ok, S, synthgen.generator(106), D=17)
        pin_product_equals_warshall(clo, mul_ok, S, synthgen.generator(107), D=13)


def test_clo_copy_passes():
    run_clo_pins(clo_ok)


@pytest.mark.parametrize("name", sorted(CLO_MUTANTS))
def test_clo_mutant_caught(name):
    with pytest.raises(AssertionError):
        run_clo_pins(CLO_MUTANTS[name])


# ---- Boolean -----------------------------------------------------------------
def bool_mul_ok(A, B, flip=False):
    """flip=True drops the k = 0 term."""
    A = np.asarray(A, np.int64)
    B = np.asarray(B, np.int64)
    P = np.zeros((A.shape[0], B.shape[1]), np.int64)
    for k in range(A.shape[1]):
        term = np.minimum(A[:, k:k + 1], B[k:k + 1, :])
        P = np.maximum(P, term) if not flip else np.maximum(P, np.maximum(A[:, k:k + 1] * 0, term) * (k > 0))
    return P


def bool_clo_ok(A, variant=None):
    T = np.asarray(A, np.int64).copy()
    D = T.shape[0]
    if variant == "reflexive":
        T = np.maximum(T, np.eye(D, dtype=np.int64))
    for k in range(D):
        row = T[k:k + 1, :] if variant != "stale_row" else np.asarray(A, np.int64)[k:k + 1, :]
        T = np.maximum(T, np.minimum(T[:, k:k + 1], row))
    return T


def test_bool_copies_pass():
    pin_bool_mul(bool_mul_ok, synthgen.generator(108))
    pin_bool_closure(bool_clo_ok, synthgen.generator(109), sizes=(1, 5, 16))


def test_bool_mutants_caught():
    with pytest.raises(AssertionError):
        pin_bool_mul(lambda A, B: bool_mul_ok(A, B, flip=True), synthgen.generator(110))
    with pytest.raises(AssertionError):  # B read transposed (square shapes only)
        pin_bool_mul(lambda A, B: bool_mul_ok(A, np.asarray(B).T)
                     if np.asarray(B).shape[0] == np.asarray(B).shape[1] else bool_mul_ok(A, B),
                     synthgen.generator(111))
    for variant in ("reflexive", "stale_row"):
        with pytest.raises(AssertionError):
            pin_bool_closure(lambda A: bool_clo_ok(A, variant), synthgen.generator(112),
                             sizes=(5, 16))
