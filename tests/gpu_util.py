"""Helpers for the GPU parity tests: seeded inputs, device copies, and the
oracle comparisons (all comparisons are bit-exact)."""
import os

import numpy as np

import oracle
import synthgen

S_OF = {1: 255, 2: 65535, 3: 255, 4: 65535, 5: 2 ** 32 - 1, 6: 2 ** 32 - 1}


def np_dtype(kind):
    return {1: np.uint8, 2: np.uint16, 3: np.uint8, 4: np.uint16, 5: np.uint32, 6: np.uint32}[kind]


def rand_dist(R, C, kind, gen, p=0.3, wmax=None):
    """Distance entries for a distance kind: present with probability p,
    distance uniform in [0, wmax], absent = S."""
    S = S_OF[kind]
    wmax = S if wmax is None else wmax
    present = gen.random((R, C)) < p
    w = gen.integers(0, wmax + 1, size=(R, C))
    return np.where(present, np.minimum(w, S), S).astype(np_dtype(kind))


def rand_antidist(R, C, kind, gen, p=0.3, wmax=None, heavy=0.0):
    """Anti-distance entries for a kind: present with probability p, distance
    uniform in [0, wmax] (default: up to S, so some saturate)."""
    S = S_OF[kind]
    wmax = S if wmax is None else wmax
    present = gen.random((R, C)) < p
    w = gen.integers(0, wmax + 1, size=(R, C))
    if heavy:
        hv = gen.random((R, C)) < heavy
        w = np.where(hv, gen.integers(S - 999 if S > 1000 else 0, S, size=(R, C)), w)
    return np.where(present & (w < S), S - w, 0).astype(np_dtype(kind))


def rand_bits(R, C, gen, p=0.1):
    return (gen.random((R, C)) < p).astype(np.uint8)


def oracle_threads():
    """Threads the oracle may use: the CPUs this process may run on, capped
    by OMP_NUM_THREADS when the machine sets it (a share of a larger host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n)


def set_oracle_threads():
    oracle.set_threads(oracle_threads())
