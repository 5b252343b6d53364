"""The C-ABI library without a GPU: it loads, exports every function that
include/semiring.h declares, and rejects bad arguments on the host before
anything is enqueued (no compute calls here)."""
import ctypes
import os
import re
import subprocess

import pytest

import paper_1705_08743_amd as sr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "semiring.h")


@pytest.fixture(scope="module")
def L():
    from paper_1705_08743_amd import build as libbuild
    if libbuild.needs_build():
        libbuild.build()
    return sr.lib()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:int64_t|int|void|char)\s*\*?\s*(\w+)\s*\(", text,
                       flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("semiring_mul", "semiring_add", "closure", "closure_batched", "sr_last_error",
              "sr_version", "sr_shutdown"):
        assert n in names
    assert set(names) == set(sr.EXPORTS)


def test_library_exports_every_declared_symbol(L):
    out = subprocess.run(["nm", "-D", "--defined-only", sr.LIB_PATH], stdout=subprocess.PIPE,
                         text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    for n in declared_functions():
        assert n in exported, n
        assert getattr(L, n) is not None


def test_version(L):
    assert "gfx950" in sr.version()


NULL = None
P = 0x7F0000000000  # 16-byte aligned fake device addresses; never dereferenced


def mul(L, kind, C, ldc, A, lda, B, ldb, R, K, N, flags=0):
    return L.semiring_mul(kind, C, ldc, A, lda, B, ldb, R, K, N, flags, None)


def test_mul_rejects_bad_arguments(L):
    U16 = sr.SR_ANTIDIST_U16
    assert mul(L, 7, P, 8, P + 4096, 8, P + 8192, 8, 4, 4, 4) == sr.SR_EINVAL
    assert "invalid kind" in L.sr_last_error().decode()
    assert mul(L, U16, P, 8, P + 4096, 8, P + 8192, 8, -1, 4, 4) == sr.SR_EINVAL
    assert mul(L, U16, P, 4, P + 4096, 8, P + 8192, 8, 4, 4, 8) == sr.SR_EINVAL  # ldc < N
    assert mul(L, U16, NULL, 8, P + 4096, 8, P + 8192, 8, 4, 4, 4) == sr.SR_EINVAL
    assert mul(L, U16, P + 2, 8, P + 4096, 8, P + 8192, 8, 4, 4, 4) == sr.SR_EALIGN
    assert mul(L, U16, P, 12, P + 4096, 8, P + 8192, 8, 4, 4, 4) == sr.SR_EALIGN  # 24-byte rows
    assert mul(L, sr.SR_ANTIDIST_U8, P, 8, P + 4096, 16, P + 8192, 16, 4, 4, 4) == sr.SR_EALIGN
    assert mul(L, sr.SR_BOOL, P, 1, P + 4096, 2, P + 8192, 2, 4, 4, 4) == sr.SR_EALIGN
    assert mul(L, U16, P, 8, P, 8, P + 8192, 8, 4, 4, 4) == sr.SR_EALIAS
    assert mul(L, U16, P, 8, P + 4096, 8, P + 16, 8, 4, 4, 4) == sr.SR_EALIAS  # partial overlap
    assert mul(L, U16, P, 8, P + 4096, 8, P + 8192, 8, 4, 4, 4, 0x100) == sr.SR_EINVAL
    # the matrix-core path is Boolean only and excludes the bitwise one
    assert mul(L, U16, P, 8, P + 4096, 8, P + 8192, 8, 4, 4, 4, sr.SR_BOOL_MFMA) == sr.SR_EINVAL
    assert mul(L, sr.SR_BOOL, P, 2, P + 4096, 2, P + 8192, 2, 4, 4, 4,
               sr.SR_BOOL_MFMA | sr.SR_BOOL_BITWISE) == sr.SR_EINVAL


def test_zero_extents_are_noops(L):
    U16 = sr.SR_ANTIDIST_U16
    assert mul(L, U16, NULL, 8, NULL, 8, P, 8, 0, 5, 5) == sr.SR_OK
    assert mul(L, U16, NULL, 8, NULL, 8, NULL, 8, 0, 5, 5) == sr.SR_EINVAL  # B is 5 x 5
    assert mul(L, U16, NULL, 8, P, 8, NULL, 8, 5, 5, 0) == sr.SR_OK
    assert L.closure(U16, NULL, 8, 0, 0, None) == sr.SR_OK
    assert L.semiring_add(U16, NULL, 8, NULL, 8, NULL, 8, 0, 0, None) == sr.SR_OK
    assert L.closure_batched(U16, None, None, None, 0, 0, None) == sr.SR_OK


def test_closure_rejects_bad_arguments(L):
    U16 = sr.SR_ANTIDIST_U16
    assert L.closure(U16, P, 8, -1, 0, None) == sr.SR_EINVAL
    assert L.closure(U16, P, 4, 8, 0, None) == sr.SR_EINVAL
    assert L.closure(U16, P + 8, 8, 8, 0, None) == sr.SR_EALIGN
    # one Boolean path at most; the matrix-core path is Boolean only
    assert L.closure(sr.SR_BOOL, P, 2, 8, sr.SR_BOOL_MFMA | sr.SR_BOOL_BITWISE,
                     None) == sr.SR_EINVAL
    assert L.closure(sr.SR_BOOL, P, 2, 8, sr.SR_BOOL_MFMA | sr.SR_BOOL_M4R, None) == sr.SR_EINVAL
    assert L.closure(U16, P, 8, 8, sr.SR_BOOL_MFMA, None) == sr.SR_EINVAL
    assert L.closure(U16, P, 8, 8, 0x400, None) == sr.SR_EINVAL
    assert L.closure(U16, P, 8, 8, sr.SR_CLOSURE_SQUARING | sr.SR_CLOSURE_WARSHALL,
                     None) == sr.SR_EINVAL
    assert L.closure(sr.SR_BOOL, P, 1, 8, 0, None) == sr.SR_EALIGN


def test_ewise_and_distance_kinds_reject_bad_arguments(L):
    f = L.semiring_ewise
    U16 = sr.SR_ANTIDIST_U16
    assert f(U16, 7, P, 8, P + 4096, 8, P + 8192, 8, 4, 4, None) == sr.SR_EINVAL
    assert "invalid op" in L.sr_last_error().decode()
    assert f(U16, -1, P, 8, P + 4096, 8, P + 8192, 8, 4, 4, None) == sr.SR_EINVAL
    assert f(9, sr.SR_EW_AND, P, 8, P + 4096, 8, P + 8192, 8, 4, 4, None) == sr.SR_EINVAL
    assert f(U16, sr.SR_EW_OR, P + 2, 8, P + 4096, 8, P + 8192, 8, 4, 4, None) == sr.SR_EALIGN
    assert f(U16, sr.SR_EW_XOR, P, 8, P + 16, 8, P + 8192, 8, 4, 4, None) == sr.SR_EALIAS
    assert f(U16, sr.SR_EW_AND, P, 8, P + 4096, 8, NULL, 8, 4, 4, None) == sr.SR_EINVAL
    assert f(U16, sr.SR_EW_NOT, NULL, 8, NULL, 8, NULL, 8, 0, 4, None) == sr.SR_OK
    for kind in (sr.SR_DISTANCE_U8, sr.SR_DISTANCE_U16):
        assert mul(L, kind, P + 1, 16, P + 4096, 16, P + 8192, 16, 4, 4, 4) == sr.SR_EALIGN
        assert L.closure(kind, P, 2, 8, 0, None) == sr.SR_EINVAL  # ld < D
        assert L.closure(kind, P, 16, 16, 0x400, None) == sr.SR_EINVAL
    assert mul(L, sr.SR_DISTANCE_U16, P, 8, P + 4096, 8, P + 8192, 8, 4, 4, 4,
               sr.SR_BOOL_MFMA) == sr.SR_EINVAL


def test_add_rejects_bad_arguments(L):
    U16 = sr.SR_ANTIDIST_U16
    f = L.semiring_add
    assert f(U16, P, 8, P + 4096, 8, P + 8192, 4, 4, 8, None) == sr.SR_EINVAL
    assert f(U16, P + 16, 8, P, 8, P + 8192, 8, 4, 8, None) == sr.SR_EALIAS  # partial overlap


def test_batched_rejects_bad_arguments(L):
    U16 = sr.SR_ANTIDIST_U16
    n = 2
    ptrs = (ctypes.c_void_p * n)(P, P + 4096)
    lds = (ctypes.c_int64 * n)(8, 8)
    dims = (ctypes.c_int64 * n)(8, 8)
    f = L.closure_batched
    assert f(9, ptrs, lds, dims, n, 0, None) == sr.SR_EINVAL  # no such kind
    # Boolean batches: ld in 64-bit words, even (16-byte rows)
    blds = (ctypes.c_int64 * n)(1, 1)
    bdims = (ctypes.c_int64 * n)(65, 65)
    assert f(sr.SR_BOOL, ptrs, blds, bdims, n, 0, None) == sr.SR_EINVAL  # 1 word < 2
    odd = (ctypes.c_int64 * n)(3, 3)
    assert f(sr.SR_BOOL, ptrs, odd, bdims, n, 0, None) == sr.SR_EALIGN  # 24-byte rows
    assert f(U16, ptrs, lds, dims, -1, 0, None) == sr.SR_EINVAL
    assert f(U16, None, lds, dims, n, 0, None) == sr.SR_EINVAL
    ptrs2 = (ctypes.c_void_p * n)(P, P + 64)  # 8 x 8 uint16 = 128 bytes: overlap
    assert f(U16, ptrs2, lds, dims, n, 0, None) == sr.SR_EALIAS
    dims2 = (ctypes.c_int64 * n)(8, 9)
    assert f(U16, ptrs, lds, dims2, n, 0, None) == sr.SR_EINVAL  # ld 8 < 9
    ptrs3 = (ctypes.c_void_p * n)(P, P + 4100)
    assert f(U16, ptrs3, lds, dims, n, 0, None) == sr.SR_EALIGN


def test_error_is_thread_local(L):
    import threading
    assert L.closure(sr.SR_ANTIDIST_U16, P, 8, -1, 0, None) == sr.SR_EINVAL
    msg_main = L.sr_last_error().decode()
    seen = {}

    def other():
        seen["msg"] = L.sr_last_error().decode()

    t = threading.Thread(target=other)
    t.start()
    t.join()
    assert seen["msg"] == "no error" and "negative" in msg_main


def test_python_binding_raises(L):
    with pytest.raises(sr.SemiringError) as ei:
        sr._check(L.closure(sr.SR_ANTIDIST_U16, P, 8, -1, 0, None))
    assert ei.value.code == sr.SR_EINVAL


def test_padded_ld():
    assert sr.padded_ld(8192, sr.SR_ANTIDIST_U16) == 8192
    assert sr.padded_ld(37, sr.SR_ANTIDIST_U16) == 64
    assert sr.padded_ld(37, sr.SR_ANTIDIST_U8) == 128
    assert sr.padded_ld(256, sr.SR_BOOL) == 16


def test_u32_kinds_validation(L):
    """32-bit kinds: 16-byte rows are multiples of 4 entries; batches are
    not built for them."""
    for kind in (sr.SR_ANTIDIST_U32, sr.SR_DISTANCE_U32):
        assert mul(L, kind, P, 6, P + 4096, 4, P + 8192, 4, 4, 4, 4) == sr.SR_EALIGN  # 24-byte rows
        assert mul(L, kind, P + 8, 4, P + 4096, 4, P + 8192, 4, 4, 4, 4) == sr.SR_EALIGN
        assert mul(L, kind, P, 4, P + 32, 4, P + 8192, 4, 4, 4, 4) == sr.SR_EALIAS  # 64-byte C
        assert mul(L, kind, P, 4, P + 4096, 4, P + 8192, 4, 4, 4, 4, sr.SR_BOOL_M4R) == sr.SR_EINVAL
        assert L.closure(kind, P, 2, 4, 0, None) == sr.SR_EINVAL  # ld < D
        assert L.closure(kind, P, 4, 4, sr.SR_BOOL_MFMA, None) == sr.SR_EINVAL
        n = 1
        ptrs = (ctypes.c_void_p * n)(P)
        lds = (ctypes.c_int64 * n)(2)
        dims = (ctypes.c_int64 * n)(4)
        assert L.closure_batched(kind, ptrs, lds, dims, n, 0, None) == sr.SR_EINVAL  # ld < D
        odd = (ctypes.c_int64 * n)(6)
        assert L.closure_batched(kind, ptrs, odd, dims, n, 0, None) == sr.SR_EALIGN
        h = ctypes.c_void_p(0)
        lds4 = (ctypes.c_int64 * n)(4)
        assert L.sr_batch_create(kind, ptrs, lds4, dims, n, 0, sr.SR_BATCH_TILE_64x16,
                                 ctypes.byref(h), None) == sr.SR_EINVAL  # one 32-bit shape
    assert sr.padded_ld(37, sr.SR_ANTIDIST_U32) == 64
    assert sr.padded_ld(37, sr.SR_DISTANCE_U32) == 64
    assert sr.elem_bytes(sr.SR_ANTIDIST_U32) == 4


def test_autotune_and_method_flags_validation(L):
    out = ctypes.c_uint(0)
    assert L.sr_autotune_closure(9, 100, ctypes.byref(out), None) == sr.SR_EINVAL
    assert L.sr_autotune_closure(sr.SR_ANTIDIST_U16, 0, ctypes.byref(out), None) == sr.SR_EINVAL
    assert L.sr_autotune_closure(sr.SR_ANTIDIST_U16, 40000, ctypes.byref(out), None) == sr.SR_EINVAL
    assert L.sr_autotune_mul(sr.SR_ANTIDIST_U16, 8, 8, 8, ctypes.byref(out), None) == sr.SR_EUNSUPPORTED
    assert L.sr_autotune_mul(sr.SR_BOOL, 0, 8, 8, ctypes.byref(out), None) == sr.SR_EINVAL
    L.sr_autotune_clear()
    U16 = sr.SR_ANTIDIST_U16
    assert L.closure(U16, P, 8, 8, sr.SR_CLOSURE_SQUARING | sr.SR_CLOSURE_BIG_BLOCKS,
                     None) == sr.SR_EINVAL
    assert L.closure(sr.SR_BOOL, P, 2, 8, sr.SR_CLOSURE_BIG_BLOCKS, None) == sr.SR_EUNSUPPORTED


def test_prepared_batch_validation(L):
    U16 = sr.SR_ANTIDIST_U16
    n = 2
    ptrs = (ctypes.c_void_p * n)(P, P + 4096)
    lds = (ctypes.c_int64 * n)(8, 8)
    dims = (ctypes.c_int64 * n)(8, 8)
    h = ctypes.c_void_p(0x1234)
    f = L.sr_batch_create
    assert f(U16, ptrs, lds, dims, n, 0, 0, None, None) == sr.SR_EINVAL  # NULL out
    assert f(U16, ptrs, lds, dims, n, 0, 4, ctypes.byref(h), None) == sr.SR_EINVAL
    assert not h.value  # cleared on every error
    assert f(U16, ptrs, lds, dims, n, 0, -1, ctypes.byref(h), None) == sr.SR_EINVAL
    assert f(sr.SR_BOOL, ptrs, lds, dims, n, sr.SR_ACCUMULATE, 0, ctypes.byref(h),
             None) == sr.SR_EINVAL
    assert f(sr.SR_ANTIDIST_U32, ptrs, lds, dims, n, 0, 3, ctypes.byref(h),
             None) == sr.SR_EINVAL  # 32-bit batches: 64 x 32 tiles only
    assert f(U16, ptrs, lds, dims, -1, 0, 0, ctypes.byref(h), None) == sr.SR_EINVAL
    assert f(U16, ptrs, lds, dims, n, sr.SR_ACCUMULATE, 0, ctypes.byref(h), None) == sr.SR_EINVAL
    ptrs2 = (ctypes.c_void_p * n)(P, P + 64)
    assert f(U16, ptrs2, lds, dims, n, 0, 0, ctypes.byref(h), None) == sr.SR_EALIAS
    assert "sr_batch_create" in L.sr_last_error().decode()
    out = ctypes.c_int(0)
    assert L.sr_batch_run(None, None) == sr.SR_EINVAL
    assert L.sr_batch_autotune(None, ctypes.byref(out), None) == sr.SR_EINVAL
    assert L.sr_batch_tile(None) == sr.SR_BATCH_TILE_AUTO
    L.sr_batch_destroy(None)
    with pytest.raises(TypeError):
        sr.PreparedBatch(U16, [])


def test_closure_noalloc_checks_before_any_device_call(L):
    """closure_noalloc validates like closure() and refuses, on the host, a
    size whose working memory exceeds its 32 MiB static scratch."""
    U16, U8 = sr.SR_ANTIDIST_U16, sr.SR_ANTIDIST_U8
    f = L.closure_noalloc
    assert f(U16, NULL, 8, 0, 0, None) == sr.SR_OK
    assert f(U16, P, 8, -1, 0, None) == sr.SR_EINVAL
    assert f(U16, P, 4, 8, 0, None) == sr.SR_EINVAL
    assert f(U16, P + 8, 8, 8, 0, None) == sr.SR_EALIGN
    assert f(U16, P, 8, 8, sr.SR_BOOL_MFMA, None) == sr.SR_EINVAL
    assert f(U16, P, 8, 8, 0x400, None) == sr.SR_EINVAL
    # uint8 data above 4096 vertices: the binary16 working copy alone is
    # 2 * D * round_up(D, 64) bytes > 32 MiB
    for kind in (U8, sr.SR_DISTANCE_U8):
        assert f(kind, P, 4112, 4100, 0, None) == sr.SR_EINVAL
        msg = L.sr_last_error().decode()
        assert "closure_noalloc" in msg and "static scratch" in msg
    # a forced squaring of a 3000-vertex uint16 matrix needs two 3000 x 3008
    # working matrices (36 MB)
    assert f(U16, P, 3008, 3000, sr.SR_CLOSURE_SQUARING, None) == sr.SR_EINVAL
    assert "static scratch" in L.sr_last_error().decode()


def test_closure_work_bytes(L):
    """The working-memory query follows closure()'s method rules: nothing for
    the 16-bit loop and for Boolean matrices, the binary16 copy for uint8
    data, two squared matrices for squaring, one big block's for big blocks,
    the transposed pivot rows for the Boolean matrix-core update; invalid
    arguments give the closure's error codes."""
    f = L.closure_work_bytes
    U16, U8 = sr.SR_ANTIDIST_U16, sr.SR_ANTIDIST_U8
    sr.autotune_clear()
    assert f(U16, 0, 0) == 0
    assert f(U16, 8192, 0) == 0
    assert f(sr.SR_BOOL, 1024, 0) == 0
    assert f(sr.SR_BOOL, 16384, sr.SR_BOOL_M4R) == 0
    # large Boolean closures update on the matrix cores by default: room for
    # the transposed pivot rows of two consecutive rounds, 32 bytes per
    # column (+ 4 words' worth) each
    assert f(sr.SR_BOOL, 16384, 0) == 2 * (16384 // 32 + 4) * 32 * 32
    assert f(U16, 600, 0) == 2 * 600 * 640 * 2 + 256                     # squaring
    assert f(U16, 2000, 0) == 2 * 512 * 512 * 2 + 256                    # big blocks
    assert f(U8, 8192, 0) == 8192 * 8192 * 2                             # binary16 copy
    assert f(U8, 600, 0) == 600 * 640 * 2 + 2 * 600 * 640 * 2 + 256
    assert f(U8, 1000, 0) == 1000 * 1024 * 2 + 2 * 512 * 512 * 2 + 256
    assert f(sr.SR_ANTIDIST_U32, 700, 0) == 2 * 700 * 704 * 4 + 256
    assert f(U16, 600, sr.SR_CLOSURE_WARSHALL) == 0
    assert f(U16, 600, sr.SR_SERIAL_PHASES) == 0
    assert f(U16, 1000, sr.SR_CLOSURE_SQUARING) == 2 * 1000 * 1024 * 2 + 256
    assert f(sr.SR_BOOL, 16384, sr.SR_BOOL_MFMA) > 0
    assert f(U16, -1, 0) == sr.SR_EINVAL
    assert f(9, 10, 0) == sr.SR_EINVAL
    assert f(U16, 10, sr.SR_BOOL_MFMA) == sr.SR_EINVAL
    assert sr.closure_work_bytes(U16, 600) == 2 * 600 * 640 * 2 + 256



def test_autotune_table_save_load(L, tmp_path):
    """The autotuning table round-trips through its JSON file, and a loaded
    entry steers closure()'s method and big-block size (seen through the
    working-memory query; without a device the architecture name is empty)."""
    U16 = sr.SR_ANTIDIST_U16
    sr.autotune_clear()
    src = tmp_path / "tune.json"
    choice_big768 = sr.SR_CLOSURE_BIG_BLOCKS | ((768 // 64) << 16)
    src.write_text('{"format": "libsemiring-autotune-1", "entries": [\n'
                   '{"arch": "", "op": 1, "kind": %d, "class": [10, 0, 0], "choice": %d},\n'
                   '{"arch": "gfx950", "op": 1, "kind": %d, "class": [9, 0, 0], "choice": %d}\n'
                   ']}\n' % (U16, choice_big768, U16, sr.SR_CLOSURE_WARSHALL))
    try:
        sr.autotune_load(str(src))
        # size class 10 = (512, 1024]: big blocks of 768 vertices
        assert sr.closure_work_bytes(U16, 1000) == 2 * 768 * 768 * 2 + 256
        # the gfx950 entry does not match this (device-less) process
        assert sr.closure_work_bytes(U16, 600) == 2 * 600 * 640 * 2 + 256
        out = tmp_path / "saved.json"
        sr.autotune_save(str(out))
        text = out.read_text()
        assert text.startswith('{"format": "libsemiring-autotune-1"')
        assert '"choice": %d' % choice_big768 in text and '"arch": "gfx950"' in text
        sr.autotune_clear()
        assert sr.closure_work_bytes(U16, 1000) == 2 * 512 * 512 * 2 + 256
        sr.autotune_load(str(out))
        assert sr.closure_work_bytes(U16, 1000) == 2 * 768 * 768 * 2 + 256
        with pytest.raises(sr.SemiringError):
            sr.autotune_load(str(tmp_path / "missing.json"))
    finally:
        sr.autotune_clear()


def test_autotune_file_environment(tmp_path):
    """With SR_AUTOTUNE_FILE set, a fresh process loads that table the first
    time the library consults it."""
    import sys
    U16 = sr.SR_ANTIDIST_U16
    f = tmp_path / "env_tune.json"
    f.write_text('{"format": "libsemiring-autotune-1", "entries": [\n'
                 '{"arch": "", "op": 1, "kind": %d, "class": [10, 0, 0], "choice": %d}\n]}\n'
                 % (U16, sr.SR_CLOSURE_BIG_BLOCKS | ((256 // 64) << 16)))
    code = ("import paper_1705_08743_amd as sr; "
            "print(sr.closure_work_bytes(sr.SR_ANTIDIST_U16, 1000))")
    env = dict(os.environ, SR_AUTOTUNE_FILE=str(f), HIP_VISIBLE_DEVICES="")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, check=True,
                         stdout=subprocess.PIPE, text=True).stdout.strip()
    assert int(out.splitlines()[-1]) == 2 * 256 * 256 * 2 + 256
