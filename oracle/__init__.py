"""CPU oracle for the semiring product and closure of arXiv 1705.08743.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product
library (``paper_1705_08743_amd``) never imports, links or calls it, and this
package never imports the product library; the two share only the seeded input
generators in ``synthgen``, which hold none of the method's arithmetic.

What it computes (all integer, so every result is exact and unique):

* Boolean semiring, Sec. II: (+) = max, (x) = min on {0, 1}.
* Anti-distance semiring, Sec. III, integer-scaled as in Sec. IV: entries
  0..S with S = 2^8 - 1 (uint8), 2^16 - 1 (uint16) or 2^32 - 1 (uint32),
  (+) = max and a (x) b = max(a + b - S, 0), evaluated in that definition
  form in int32 (int64 for S = 2^32 - 1).
* ``mul``:     the multiplication algorithm of Sec. II (P := 0, then for every
               k, P := P (+) column k of A times row k of B).
* ``closure``: Warshall's algorithm of Sec. II (T := A, then for every k,
               T := T (+) column k of T times row k of T, in place), i.e. the
               transitive, non-reflexive closure A (+) A*A (+) ... (eq. trcl).
* ``closure_rows``: selected rows of that closure straight from its path
               definition (Dijkstra on distances S - entry, or breadth-first
               search for Boolean), for sampled checks at sizes where the full
               Warshall loop is too slow.
* ``add``:     entrywise (+) (Sec. II; the | operator of the table of entrywise
               operations in Sec. V).
* ``ewise``:   the entrywise operations of that table: and = min, or = max,
               xor = |a - b|, not = S - a (on Boolean words: AND, OR, XOR, NOT
               with the padding bits kept zero).
* ``dist_mul``, ``dist_closure``: the distance-matrix dual the paper adds
               (addition min, multiplication saturating +, S = no path), by
               the same multiplication algorithm and Warshall loop.
* ``reflexive``: I (+) T (eq. rtc), the multiplicative identity's diagonal
               (S for anti-distance, 1 for Boolean, 0 for distance) added in.

Every function here is pinned by the ``-m "not gpu"`` tests in
``tests/test_oracle_pins.py`` against brute force, closed forms, invariants and
library routines that share nothing with this code.

Boolean matrices cross this interface either unpacked (uint8 arrays of 0/1) or
bit-packed (uint64 words, entry (r, c) at bit c % 64 of word c // 64 of row r,
the least-significant-bit-first order of the paper's Boolean listing, Sec. IV).
"""
import ctypes
import os

import numpy as np

from . import build as _build

S_U8 = 2 ** 8 - 1
S_U16 = 2 ** 16 - 1
S_U32 = 2 ** 32 - 1

_lib = None


def _load():
    global _lib
    if _lib is None:
        path = _build.ensure_built()
        lib = ctypes.CDLL(path)
        i64, i32, vp = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p
        lib.o_set_threads.argtypes = [ctypes.c_int]
        lib.o_get_max_threads.restype = ctypes.c_int
        lib.o_has_openmp.restype = ctypes.c_int
        lib.o_ad_mul.argtypes = [vp, i64, vp, i64, vp, i64, i64, i64, i64, i32, ctypes.c_int]
        lib.o_ad_closure_steps.argtypes = [vp, i64, i64, i32, i64, i64]
        lib.o_ad_closure.argtypes = [vp, i64, i64, i32]
        lib.o_ad_closure_rows.argtypes = [vp, i64, i64, i32, vp, i64, vp]
        lib.o_bool_mul.argtypes = [vp, i64, vp, i64, vp, i64, i64, i64, i64, ctypes.c_int]
        lib.o_bool_closure.argtypes = [vp, i64, i64]
        lib.o_bool_mul_words.argtypes = [vp, i64, vp, i64, vp, i64, i64, i64, i64, ctypes.c_int]
        lib.o_bool_closure_words.argtypes = [vp, i64, i64]
        lib.o_bool_closure_rows_words.argtypes = [vp, i64, i64, vp, i64, vp, i64]
        lib.o_dist_mul.argtypes = [vp, i64, vp, i64, vp, i64, i64, i64, i64, i32, ctypes.c_int]
        lib.o_dist_closure.argtypes = [vp, i64, i64, i32]
        lib.o_ad_mul64.argtypes = [vp, i64, vp, i64, vp, i64, i64, i64, i64, i64, ctypes.c_int]
        lib.o_ad_closure_steps64.argtypes = [vp, i64, i64, i64, i64, i64]
        lib.o_dist_mul64.argtypes = [vp, i64, vp, i64, vp, i64, i64, i64, i64, i64, ctypes.c_int]
        lib.o_dist_closure64.argtypes = [vp, i64, i64, i64]
        lib.o_ad_closure_rows64.argtypes = [vp, i64, i64, i64, vp, i64, vp]
        _lib = lib
    return _lib


def set_threads(n: int) -> None:
    """Threads for the i-loop inside one k step (results do not depend on it)."""
    _load().o_set_threads(int(n))


def max_threads() -> int:
    return int(_load().o_get_max_threads())


def has_openmp() -> bool:
    return bool(_load().o_has_openmp())


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def scale(dtype) -> int:
    """S for an unsigned storage type (Sec. IV: 2^8-1, 2^16-1)."""
    dtype = np.dtype(dtype)
    if dtype == np.uint8:
        return S_U8
    if dtype == np.uint16:
        return S_U16
    if dtype == np.uint32:
        return S_U32
    raise ValueError("anti-distance entries are uint8, uint16 or uint32, got %s" % dtype)


def _as_i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _as_i64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


def _wide(S):
    """S = 2^32 - 1 needs the int64 loops (a + b does not fit in int32)."""
    return int(S) > 2 ** 31 - 1


# --------------------------------------------------------------------------
# anti-distance
# --------------------------------------------------------------------------
def ad_mul(A, B, S, C=None):
    """(A * B) over the anti-distance semiring; with C given, C (+) A * B.

    A: R x K, B: K x N, entries in 0..S (any integer dtype).  Returns int32."""
    wide = _wide(S)
    conv = _as_i64 if wide else _as_i32
    A = conv(A)
    B = conv(B)
    R, K = A.shape
    K2, N = B.shape
    if K != K2:
        raise ValueError("inner dimensions differ: %d vs %d" % (K, K2))
    acc = C is not None
    out = conv(C).copy() if acc else np.zeros((R, N), np.int64 if wide else np.int32)
    if R and N:
        f = _load().o_ad_mul64 if wide else _load().o_ad_mul
        f(_ptr(A), K, _ptr(B), N, _ptr(out), N, R, K, N, int(S), int(acc))
    return out


def ad_closure(A, S, k_end=None):
    """Warshall/Floyd closure over the anti-distance semiring (int32 result).

    With k_end given, only the first k_end pivot steps are run (used to time a
    bounded sample of the full loop)."""
    wide = _wide(S)
    T = (_as_i64 if wide else _as_i32)(A).copy()
    D = T.shape[0]
    if T.shape != (D, D):
        raise ValueError("closure needs a square matrix")
    k1 = D if k_end is None else int(k_end)
    if D:
        f = _load().o_ad_closure_steps64 if wide else _load().o_ad_closure_steps
        f(_ptr(T), D, D, int(S), 0, k1)
    return T


def ad_closure_rows(A, S, rows):
    """Rows ``rows`` of the anti-distance closure from its path definition."""
    wide = _wide(S)
    A = (_as_i64 if wide else _as_i32)(A)
    D = A.shape[0]
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.zeros((len(rows), D), np.int64 if wide else np.int32)
    if len(rows) and D:
        f = _load().o_ad_closure_rows64 if wide else _load().o_ad_closure_rows
        f(_ptr(A), D, D, int(S), _ptr(rows), len(rows), _ptr(out))
    return out


def ad_add(A, B):
    """Entrywise (+) = max (Sec. II matrix addition)."""
    return np.maximum(_as_i32(A), _as_i32(B))


# --------------------------------------------------------------------------
# distance matrices (the dual: min, saturating +)
# --------------------------------------------------------------------------
def dist_mul(A, B, S, C=None):
    """Distance product: min over k of min(A_ik + B_kj, S); with C given,
    min(C, A + B).  Entries 0..S, S = no path.  Returns int32."""
    wide = _wide(S)
    conv = _as_i64 if wide else _as_i32
    A = conv(A)
    B = conv(B)
    R, K = A.shape
    K2, N = B.shape
    if K != K2:
        raise ValueError("inner dimensions differ: %d vs %d" % (K, K2))
    acc = C is not None
    out = conv(C).copy() if acc else np.full((R, N), int(S), np.int64 if wide else np.int32)
    if R and N:
        f = _load().o_dist_mul64 if wide else _load().o_dist_mul
        f(_ptr(A), K, _ptr(B), N, _ptr(out), N, R, K, N, int(S), int(acc))
    return out


def dist_closure(A, S):
    """Warshall's loop with min and saturating + (distance closure; the
    diagonal holds the shortest cycle through each vertex, or S)."""
    wide = _wide(S)
    T = (_as_i64 if wide else _as_i32)(A).copy()
    D = T.shape[0]
    if T.shape != (D, D):
        raise ValueError("closure needs a square matrix")
    if D:
        f = _load().o_dist_closure64 if wide else _load().o_dist_closure
        f(_ptr(T), D, D, int(S))
    return T


# --------------------------------------------------------------------------
# entrywise operations (table of Sec. V) and the reflexive closure (eq. rtc)
# --------------------------------------------------------------------------
def ewise(op, A, B=None, S=None):
    """Entrywise and = min, or = max, xor = |a - b|, not = S - a (int64)."""
    A = np.asarray(A, np.int64)
    if op == "not":
        return int(S) - A
    B = np.asarray(B, np.int64)
    if op == "and":
        return np.minimum(A, B)
    if op == "or":
        return np.maximum(A, B)
    if op == "xor":
        return np.abs(A - B)
    raise ValueError("op is and, or, xor or not")


def ewise_words(op, A, N, B=None):
    """The same operations on bit-packed Boolean rows of N bits (AND, OR, XOR,
    NOT); padding bits of the result are zero."""
    A = _as_words(A)
    if op == "not":
        out = ~A
    elif op == "and":
        out = A & _as_words(B)
    elif op == "or":
        out = A | _as_words(B)
    elif op == "xor":
        out = A ^ _as_words(B)
    else:
        raise ValueError("op is and, or, xor or not")
    out = out.copy()
    nw = (N + 63) // 64
    out[:, nw:] = 0
    if N % 64:
        out[:, nw - 1] &= np.uint64((1 << (N % 64)) - 1)
    return out


def reflexive(T, one):
    """I (+) T: the diagonal combined with the multiplicative identity `one`
    (anti-distance: max with S; Boolean: max with 1; distance: min with 0)."""
    out = np.array(T, copy=True)
    d = np.arange(min(out.shape))
    if one == 0:
        out[d, d] = np.minimum(out[d, d], 0)
    else:
        out[d, d] = np.maximum(out[d, d], one)
    return out


# --------------------------------------------------------------------------
# Boolean, unpacked {0,1} bytes
# --------------------------------------------------------------------------
def _as_u8(a):
    a = np.ascontiguousarray(a, dtype=np.uint8)
    if a.size and a.max() > 1:
        raise ValueError("Boolean entries must be 0 or 1")
    return a


def bool_mul(A, B, C=None):
    A = _as_u8(A)
    B = _as_u8(B)
    R, K = A.shape
    K2, N = B.shape
    if K != K2:
        raise ValueError("inner dimensions differ: %d vs %d" % (K, K2))
    acc = C is not None
    out = _as_u8(C).copy() if acc else np.zeros((R, N), np.uint8)
    if R and N:
        _load().o_bool_mul(_ptr(A), K, _ptr(B), N, _ptr(out), N, R, K, N, int(acc))
    return out


def bool_closure(A):
    T = _as_u8(A).copy()
    D = T.shape[0]
    if T.shape != (D, D):
        raise ValueError("closure needs a square matrix")
    if D:
        _load().o_bool_closure(_ptr(T), D, D)
    return T


def bool_add(A, B):
    return np.maximum(_as_u8(A), _as_u8(B))


# --------------------------------------------------------------------------
# Boolean, bit-packed uint64 words
# --------------------------------------------------------------------------
def _as_words(a):
    return np.ascontiguousarray(a, dtype=np.uint64)


def bool_mul_words(A, B, K, N, C=None):
    """Packed Boolean product.  A: R x ldA words holding R x K bits; B: K x
    ldB words holding K x N bits.  Returns R x ceil(N/64) words (or C's shape
    when accumulating into C)."""
    A = _as_words(A)
    B = _as_words(B)
    R = A.shape[0]
    if B.shape[0] != K:
        raise ValueError("B must have K rows")
    nw = (N + 63) // 64
    acc = C is not None
    out = _as_words(C).copy() if acc else np.zeros((R, nw), np.uint64)
    if R and N:
        _load().o_bool_mul_words(_ptr(A), A.shape[1], _ptr(B), B.shape[1], _ptr(out),
                                 out.shape[1], R, K, N, int(acc))
    return out


def bool_closure_words(A, D):
    T = _as_words(A).copy()
    if T.shape[0] != D:
        raise ValueError("closure needs D rows")
    if D:
        _load().o_bool_closure_words(_ptr(T), T.shape[1], D)
    return T


def bool_closure_rows_words(A, D, rows):
    A = _as_words(A)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    nw = (D + 63) // 64
    out = np.zeros((len(rows), nw), np.uint64)
    if len(rows) and D:
        _load().o_bool_closure_rows_words(_ptr(A), A.shape[1], D, _ptr(rows), len(rows),
                                          _ptr(out), nw)
    return out


def bool_add_words(A, B):
    return np.bitwise_or(_as_words(A), _as_words(B))


__all__ = [
    "S_U8", "S_U16", "scale", "set_threads", "max_threads", "has_openmp",
    "ad_mul", "ad_closure", "ad_closure_rows", "ad_add",
    "bool_mul", "bool_closure", "bool_add",
    "bool_mul_words", "bool_closure_words", "bool_closure_rows_words", "bool_add_words",
]
