"""Python binding of libsemiring, the gfx950 implementation of the semiring
product and closure of de Bondt, arXiv 1705.08743 (see include/semiring.h).

Argument marshalling only: every step runs in the HIP kernels of
``libsemiring.so``; torch supplies device memory and the current stream.  The
functions mirror the C ABI names and raise ``SemiringError`` on a non-zero
return.  If the library has not been built, the first call raises: there is no
fallback.

Matrices are 2-D CUDA (HIP) tensors with unit column stride; the row stride
``tensor.stride(0)`` is the ABI's leading dimension ``ld``:

* anti-distance (``SR_ANTIDIST_U8`` / ``_U16`` / ``_U32``) and distance
  (``SR_DISTANCE_U8`` / ``_U16`` / ``_U32``): ``torch.uint8`` /
  ``torch.uint16`` / ``torch.uint32`` tensors; the logical shape is the tensor
  shape, so a view ``X[:, :n]`` of a padded ``(rows, ld)`` buffer is a
  rows x n matrix.
* Boolean (``SR_BOOL``): ``torch.int64`` tensors of packed words (entry (r, c)
  at bit c % 64 of word c // 64, least significant bit first); bit widths are
  passed explicitly (``K``, ``N``, ``D``) and default to 64 x words.
"""
import ctypes
import os

SR_BOOL = 0
SR_ANTIDIST_U8 = 1
SR_ANTIDIST_U16 = 2
SR_DISTANCE_U8 = 3
SR_DISTANCE_U16 = 4
SR_ANTIDIST_U32 = 5
SR_DISTANCE_U32 = 6

SR_EW_AND = 0
SR_EW_OR = 1
SR_EW_XOR = 2
SR_EW_NOT = 3

_U8_KINDS = (SR_ANTIDIST_U8, SR_DISTANCE_U8)
_U16_KINDS = (SR_ANTIDIST_U16, SR_DISTANCE_U16)
_U32_KINDS = (SR_ANTIDIST_U32, SR_DISTANCE_U32)


def elem_bytes(kind):
    """Bytes per stored entry (8 for Boolean words)."""
    if kind in _U8_KINDS:
        return 1
    if kind in _U16_KINDS:
        return 2
    if kind in _U32_KINDS:
        return 4
    return 8

SR_OK = 0
SR_EINVAL = -1
SR_EALIAS = -2
SR_EALIGN = -3
SR_ENOMEM = -4
SR_EDEVICE = -5
SR_EUNSUPPORTED = -6

SR_ACCUMULATE = 1
SR_REFLEXIVE = 2
SR_BOOL_BITWISE = 4
SR_BOOL_MFMA = 8
SR_SERIAL_PHASES = 16
SR_BOOL_M4R = 32
SR_CLOSURE_SQUARING = 64
SR_CLOSURE_WARSHALL = 128
SR_CLOSURE_BIG_BLOCKS = 256

# update-tile shapes of a prepared batch (entries per wave tile)
SR_BATCH_TILE_AUTO = 0
SR_BATCH_TILE_64x16 = 1
SR_BATCH_TILE_64x32 = 2
SR_BATCH_TILE_64x64 = 3

ERROR_NAMES = {
    SR_EINVAL: "SR_EINVAL", SR_EALIAS: "SR_EALIAS", SR_EALIGN: "SR_EALIGN",
    SR_ENOMEM: "SR_ENOMEM", SR_EDEVICE: "SR_EDEVICE", SR_EUNSUPPORTED: "SR_EUNSUPPORTED",
}

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsemiring.so")

EXPORTS = ("semiring_mul", "semiring_add", "semiring_ewise", "closure", "closure_work_bytes",
           "closure_noalloc",
           "closure_batched",
           "sr_autotune_closure", "sr_autotune_mul", "sr_autotune_clear", "sr_autotune_save",
           "sr_autotune_load",
           "sr_batch_create", "sr_batch_run", "sr_batch_autotune", "sr_batch_tile",
           "sr_batch_destroy",
           "sr_profile_enable", "sr_profile_read", "sr_last_error", "sr_version", "sr_shutdown")

SR_PHASE_PIVOT = 0
SR_PHASE_PANELS = 1
SR_PHASE_UPDATE = 2


class SemiringError(RuntimeError):
    def __init__(self, code, message):
        super().__init__("%s (%d): %s" % (ERROR_NAMES.get(code, "error"), code, message))
        self.code = code


_lib = None


def lib():
    """The loaded library (ctypes); raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                "libsemiring.so is not built (expected at %s); run "
                "`python -c 'import __graft_entry__ as g; g.build()'` or "
                "`python paper_1705_08743_amd/build.py`" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        i64, vp, u32, i32 = ctypes.c_int64, ctypes.c_void_p, ctypes.c_uint, ctypes.c_int
        L.semiring_mul.argtypes = [i32, vp, i64, vp, i64, vp, i64, i64, i64, i64, u32, vp]
        L.semiring_mul.restype = i32
        L.semiring_add.argtypes = [i32, vp, i64, vp, i64, vp, i64, i64, i64, vp]
        L.semiring_add.restype = i32
        L.semiring_ewise.argtypes = [i32, i32, vp, i64, vp, i64, vp, i64, i64, i64, vp]
        L.semiring_ewise.restype = i32
        L.closure.argtypes = [i32, vp, i64, i64, u32, vp]
        L.closure.restype = i32
        L.closure_noalloc.argtypes = [i32, vp, i64, i64, u32, vp]
        L.closure_noalloc.restype = i32
        L.closure_work_bytes.argtypes = [i32, i64, u32]
        L.closure_work_bytes.restype = i64
        L.closure_batched.argtypes = [i32, ctypes.POINTER(vp), ctypes.POINTER(i64),
                                      ctypes.POINTER(i64), i64, u32, vp]
        L.closure_batched.restype = i32
        L.sr_autotune_closure.argtypes = [i32, i64, ctypes.POINTER(u32), vp]
        L.sr_autotune_closure.restype = i32
        L.sr_autotune_mul.argtypes = [i32, i64, i64, i64, ctypes.POINTER(u32), vp]
        L.sr_autotune_mul.restype = i32
        L.sr_autotune_clear.restype = None
        L.sr_autotune_save.argtypes = [ctypes.c_char_p]
        L.sr_autotune_save.restype = i32
        L.sr_autotune_load.argtypes = [ctypes.c_char_p]
        L.sr_autotune_load.restype = i32
        L.sr_batch_create.argtypes = [i32, ctypes.POINTER(vp), ctypes.POINTER(i64),
                                      ctypes.POINTER(i64), i64, u32, i32,
                                      ctypes.POINTER(vp), vp]
        L.sr_batch_create.restype = i32
        L.sr_batch_run.argtypes = [vp, vp]
        L.sr_batch_run.restype = i32
        L.sr_batch_autotune.argtypes = [vp, ctypes.POINTER(i32), vp]
        L.sr_batch_autotune.restype = i32
        L.sr_batch_tile.argtypes = [vp]
        L.sr_batch_tile.restype = i32
        L.sr_batch_destroy.argtypes = [vp]
        L.sr_batch_destroy.restype = None
        L.sr_last_error.restype = ctypes.c_char_p
        L.sr_version.restype = ctypes.c_char_p
        L.sr_shutdown.restype = None
        L.sr_profile_enable.argtypes = [i32]
        L.sr_profile_enable.restype = i32
        L.sr_profile_read.argtypes = [i32, i32, ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_double)]
        L.sr_profile_read.restype = i32
        _lib = L
    return _lib


def _check(rc):
    if rc != SR_OK:
        raise SemiringError(rc, lib().sr_last_error().decode())


_TORCH = None


def _torch():
    global _TORCH
    if _TORCH is None:
        import torch
        _TORCH = torch
    return _TORCH


_DTYPE_KIND = None


def kind_of(t):
    """Semiring kind implied by a tensor's dtype."""
    torch = _torch()
    if t.dtype == torch.uint8:
        return SR_ANTIDIST_U8
    if t.dtype == torch.uint16:
        return SR_ANTIDIST_U16
    if t.dtype == torch.uint32:
        return SR_ANTIDIST_U32
    if t.dtype == torch.int64:
        return SR_BOOL
    raise TypeError("unsupported dtype %s (uint8, uint16, uint32 or int64 words)" % t.dtype)


def _mat(t, name):
    """(data pointer or None, row stride, rows, cols) of a 2-D device tensor
    with unit column stride.  Few tensor attribute reads: at the smallest
    sizes this marshalling is a visible part of a call's latency."""
    if t is None:
        return None, 0, 0, 0
    shape, stride = t.shape, t.stride()
    if len(shape) != 2:
        raise ValueError("%s must be a 2-D tensor" % name)
    r, c = shape
    s0, s1 = stride
    ld = s0 if r > 1 else max(s0, c)
    if not (r and c):
        return None, ld, r, c
    if s1 != 1:
        raise ValueError("%s must have unit column stride" % name)
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    return t.data_ptr(), ld, r, c


def _stream(stream):
    """The HIP stream handle (an int; 0 is the null stream): torch's current
    stream of the current device when stream is None."""
    if stream is None:
        C = _torch()._C
        raw = getattr(C, "_cuda_getCurrentRawStream", None)
        if raw is not None:
            return raw(C._cuda_getDevice())
        return _torch().cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def semiring_mul(kind, C, A, B, R=None, K=None, N=None, flags=0, stream=None):
    """C := A * B, or C (+)= A * B with flags=SR_ACCUMULATE (in place on C)."""
    pc, ldc, rc_, nc = _mat(C, "C")
    pa, lda, ra, ka = _mat(A, "A")
    pb, ldb, rb, nb = _mat(B, "B")
    if kind == SR_BOOL:
        R = ra if R is None else R
        K = 64 * ka if K is None else K
        N = 64 * nc if N is None else N
    else:
        R = ra if R is None else R
        K = ka if K is None else K
        N = nb if N is None else N
    _check(lib().semiring_mul(kind, pc, ldc, pa, lda, pb, ldb, R, K, N, flags, _stream(stream)))


def semiring_add(kind, C, A, B, R=None, N=None, stream=None):
    """C := A (+) B entrywise (C may be A or B)."""
    pc, ldc, _, nc = _mat(C, "C")
    pa, lda, ra, na = _mat(A, "A")
    pb, ldb, _, _ = _mat(B, "B")
    R = ra if R is None else R
    N = (64 * nc if kind == SR_BOOL else na) if N is None else N
    _check(lib().semiring_add(kind, pc, ldc, pa, lda, pb, ldb, R, N, _stream(stream)))


def semiring_ewise(kind, op, C, A, B=None, R=None, N=None, stream=None):
    """C := A op B entrywise (op = SR_EW_AND, SR_EW_OR, SR_EW_XOR), or
    C := not A (SR_EW_NOT, B unused); C may be A or B."""
    pc, ldc, _, nc = _mat(C, "C")
    pa, lda, ra, na = _mat(A, "A")
    pb, ldb = (None, 0) if B is None else _mat(B, "B")[:2]
    R = ra if R is None else R
    N = (64 * nc if kind == SR_BOOL else na) if N is None else N
    _check(lib().semiring_ewise(kind, op, pc, ldc, pa, lda, pb, ldb, R, N, _stream(stream)))


def closure(kind, T, D=None, flags=0, stream=None):
    """In-place transitive closure of the D x D matrix held in T."""
    pt, ldt, rt, ct = _mat(T, "T")
    D = rt if D is None else D
    _check(lib().closure(kind, pt, ldt, D, flags, _stream(stream)))


def closure_work_bytes(kind, D, flags=0):
    """Device bytes closure(kind, D, flags) would allocate for its duration."""
    n = lib().closure_work_bytes(kind, D, flags)
    if n < 0:
        _check(int(n))
    return int(n)


def closure_noalloc(kind, T, D=None, flags=0, stream=None):
    """closure() without allocation: working memory from the library's static
    per-device scratch (32 MiB); raises SemiringError (SR_EINVAL) for sizes
    whose working memory does not fit."""
    pt, ldt, rt, ct = _mat(T, "T")
    D = rt if D is None else D
    _check(lib().closure_noalloc(kind, pt, ldt, D, flags, _stream(stream)))


def closure_batched(kind, Ts, Ds=None, flags=0, stream=None):
    """In-place closures of every matrix of a batch (one call): Ts is a list
    of square matrix tensors, or a BatchArena (whose argument arrays are
    built once, so a call costs no per-matrix Python work)."""
    if isinstance(Ts, BatchArena):
        if Ds is not None:
            raise ValueError("a BatchArena carries its own sizes")
        a = Ts
        _check(lib().closure_batched(kind, a._ptrs_c, a._lds_c, a._dims_c, a.count, flags,
                                     _stream(stream)))
        return
    n = len(Ts)
    ptrs = (ctypes.c_void_p * n)()
    lds = (ctypes.c_int64 * n)()
    dims = (ctypes.c_int64 * n)()
    for i, t in enumerate(Ts):
        p, ld, r, _ = _mat(t, "T[%d]" % i)
        ptrs[i] = p
        lds[i] = ld
        dims[i] = r if Ds is None else Ds[i]
    _check(lib().closure_batched(kind, ptrs, lds, dims, n, flags, _stream(stream)))


class BatchArena:
    """A batch of square matrices back to back in one device buffer: matrix i
    (sizes[i] vertices) starts at a 256-byte aligned offset and has a row
    stride of padded_ld(sizes[i]) entries (Boolean: ceil(sizes[i] / 64)
    64-bit words rounded up to an even count).  The pointer, stride and size
    arrays that closure_batched passes to the C ABI are built once here, with
    numpy, so repeated calls on the same batch do no per-matrix marshalling.
    The arena owns its buffer (``self.buf``, a flat uint8 tensor): the
    pointers stay valid while the arena is alive."""

    def __init__(self, kind, sizes, device="cuda", zero=True):
        import numpy as np
        torch = _torch()
        if kind not in _U8_KINDS + _U16_KINDS + _U32_KINDS + (SR_BOOL,):
            raise ValueError("BatchArena holds Boolean, anti-distance or distance matrices")
        self.kind = kind
        self.es = {SR_BOOL: 8}.get(kind, 1 if kind in _U8_KINDS else
                                   (4 if kind in _U32_KINDS else 2))
        self.dtype = {1: torch.uint8, 2: torch.uint16, 4: torch.uint32, 8: torch.int64}[self.es]
        self.sizes = np.asarray(sizes, dtype=np.int64).reshape(-1)
        if (self.sizes < 0).any():
            raise ValueError("negative matrix size")
        self.count = int(self.sizes.size)
        if kind == SR_BOOL:
            # words per row, even (16-byte rows)
            self.lds = np.maximum(2, -(-(-(-self.sizes // 64)) // 2) * 2).astype(np.int64)
        else:
            per = 128 // self.es
            self.lds = np.maximum(per, -(-self.sizes // per) * per).astype(np.int64)
        nbytes = -(-(self.sizes * self.lds * self.es) // 256) * 256
        self.offsets = np.zeros(self.count, dtype=np.int64)
        if self.count > 1:
            self.offsets[1:] = np.cumsum(nbytes)[:-1]
        total = int(nbytes.sum()) if self.count else 0
        self.buf = (torch.zeros if zero else torch.empty)(max(total, 256), dtype=torch.uint8,
                                                           device=device)
        self._ptrs = (self.buf.data_ptr() + self.offsets).astype(np.int64)
        self._dims = self.sizes.copy()
        self._ptrs_c = self._ptrs.ctypes.data_as(ctypes.POINTER(ctypes.c_void_p))
        self._lds_c = self.lds.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        self._dims_c = self._dims.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))

    def __len__(self):
        return self.count

    def _width(self, n):
        """Stored units of a row of an n-vertex matrix (entries, or words)."""
        return -(-n // 64) if self.kind == SR_BOOL else n

    def view(self, i):
        """Matrix i as a tensor view of sizes[i] rows (row stride lds[i]):
        sizes[i] entries per row, or ceil(sizes[i] / 64) int64 words."""
        n, ld, off = int(self.sizes[i]), int(self.lds[i]), int(self.offsets[i])
        flat = self.buf[off:off + n * ld * self.es].view(self.dtype)
        return flat.view(n, ld)[:, :self._width(n)]

    def host_image(self, mats):
        """The arena's bytes (numpy uint8) with the host matrices `mats`
        (entries, or uint64 words for Boolean) in place, padding zero."""
        import numpy as np
        img = np.zeros(self.buf.numel(), dtype=np.uint8)
        np_dt = {1: np.uint8, 2: np.uint16, 4: np.uint32, 8: np.uint64}[self.es]
        for i, m in enumerate(mats):
            n, ld, off = int(self.sizes[i]), int(self.lds[i]), int(self.offsets[i])
            w = self._width(n)
            if m.shape[0] != n or m.shape[1] < w:
                raise ValueError("matrix %d has shape %s, expected %d x %d" % (i, m.shape, n, w))
            dst = img[off:off + n * ld * self.es].view(np_dt).reshape(n, ld)
            dst[:, :w] = m[:, :w]
        return img

    def load(self, mats):
        """Copy host matrices into the arena (one host-to-device copy)."""
        torch = _torch()
        self.buf.copy_(torch.from_numpy(self.host_image(mats)))

    def copy_(self, other):
        """Copy another arena of the same layout (one device copy)."""
        import numpy as np
        if self.kind != other.kind or not np.array_equal(self.sizes, other.sizes):
            raise ValueError("arena layouts differ")
        self.buf.copy_(other.buf)


class PreparedBatch:
    """A batch prepared once for repeated closures (sr_batch_create): ``run()``
    enqueues kernel launches only, so it can be captured into a CUDA/HIP graph
    (``torch.cuda.CUDAGraph``) and the whole batch closed by one replay.
    ``arena`` is a BatchArena (kept alive by this object); tile is one of the
    SR_BATCH_TILE_* shapes.  ``close()`` frees the device plan; a graph that
    captured ``run()`` must not be replayed after that."""

    def __init__(self, kind, arena, flags=0, tile=SR_BATCH_TILE_AUTO, stream=None):
        if not isinstance(arena, BatchArena):
            raise TypeError("PreparedBatch takes a BatchArena")
        self.kind = kind
        self.arena = arena
        self._h = ctypes.c_void_p(None)
        _check(lib().sr_batch_create(kind, arena._ptrs_c, arena._lds_c, arena._dims_c,
                                     arena.count, flags, tile, ctypes.byref(self._h),
                                     _stream(stream)))

    def _handle(self):
        if not self._h:
            raise ValueError("the prepared batch has been closed")
        return self._h

    def run(self, stream=None):
        """In-place closure of the arena's current contents."""
        _check(lib().sr_batch_run(self._handle(), _stream(stream)))

    def autotune(self, stream=None):
        """Time the update-tile shapes, keep the fastest; returns its code."""
        out = ctypes.c_int(0)
        _check(lib().sr_batch_autotune(self._handle(), ctypes.byref(out), _stream(stream)))
        return out.value

    @property
    def tile(self):
        return lib().sr_batch_tile(self._handle())

    def close(self):
        if self._h:
            lib().sr_batch_destroy(self._h)
            self._h = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune_closure(kind, D, stream=None):
    """Time the closure methods for (kind, D) and keep the fastest for D's
    size class; returns its flags (SR_CLOSURE_* [| SR_BOOL_*])."""
    out = ctypes.c_uint(0)
    _check(lib().sr_autotune_closure(kind, D, ctypes.byref(out), _stream(stream)))
    return out.value


def autotune_mul(kind, R, K, N, stream=None):
    """Time the Boolean product paths for (R, K, N) and keep the fastest for
    its size class; returns its flag (SR_BOOL_BITWISE / _M4R / _MFMA)."""
    out = ctypes.c_uint(0)
    _check(lib().sr_autotune_mul(kind, R, K, N, ctypes.byref(out), _stream(stream)))
    return out.value


def autotune_save(path):
    """Write the autotuning table to `path` (JSON)."""
    _check(lib().sr_autotune_save(os.fsencode(path)))


def autotune_load(path):
    """Merge the autotuning table saved at `path`."""
    _check(lib().sr_autotune_load(os.fsencode(path)))


def autotune_clear():
    """Forget every autotuned choice."""
    lib().sr_autotune_clear()


def version():
    return lib().sr_version().decode()


def sr_profile_enable(enable=True):
    """Start (or stop) recording hipEvents around each closure phase launch."""
    _check(lib().sr_profile_enable(1 if enable else 0))


def sr_profile_read(kind, phase):
    """(total_ms, launches, updates) of the recorded launches of one phase."""
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    u = ctypes.c_double()
    _check(lib().sr_profile_read(kind, phase, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(u)))
    return ms.value, n.value, u.value


def shutdown():
    lib().sr_shutdown()


# ---------------------------------------------------------------------------
# allocation helpers (device memory comes from torch)
# ---------------------------------------------------------------------------
def padded_ld(cols, kind, align_bytes=128):
    """Row stride (elements, or words for Boolean) for `cols` columns, rounded
    to `align_bytes` (128 bytes lets every wave tile take the wide path)."""
    if kind == SR_BOOL:
        words = (cols + 63) // 64
        per = max(2, align_bytes // 8)
        return max(per, -(-words // per) * per)
    per = align_bytes // elem_bytes(kind)
    return max(per, -(-cols // per) * per)


def empty(kind, rows, cols, device="cuda", zero=True):
    """A rows x cols matrix view of a zero-filled padded device buffer (for
    Boolean, rows x words with cols bits of payload)."""
    torch = _torch()
    dt = {SR_BOOL: torch.int64, SR_ANTIDIST_U8: torch.uint8, SR_ANTIDIST_U16: torch.uint16,
          SR_DISTANCE_U8: torch.uint8, SR_DISTANCE_U16: torch.uint16,
          SR_ANTIDIST_U32: torch.uint32, SR_DISTANCE_U32: torch.uint32}[kind]
    ld = padded_ld(cols, kind)
    buf = (torch.zeros if zero else torch.empty)((max(rows, 1), ld), dtype=dt, device=device)
    width = (cols + 63) // 64 if kind == SR_BOOL else cols
    return buf[:rows, :width]


def clone(t):
    """A copy of a matrix view with the same row stride (torch's clone of a
    padded view would drop the padding and could break row alignment)."""
    torch = _torch()
    rows, cols = t.shape
    ld = t.stride(0) if rows > 1 else max(t.stride(0), cols)
    buf = torch.empty((max(rows, 1), ld), dtype=t.dtype, device=t.device)
    out = buf[:rows, :cols]
    out.copy_(t)
    return out


def to_device(kind, host, cols=None, device="cuda"):
    """Copy a host numpy matrix (uint8 / uint16 / uint32 entries, or uint64 words) into
    a padded device buffer; returns the logical view."""
    import numpy as np
    torch = _torch()
    host = np.ascontiguousarray(host)
    rows = host.shape[0]
    if kind == SR_BOOL:
        words = host.shape[1] if cols is None else (cols + 63) // 64
        cols = 64 * words if cols is None else cols
        out = empty(kind, rows, cols, device)
        out.copy_(torch.from_numpy(host[:, :words].view(np.int64)))
        return out
    cols = host.shape[1] if cols is None else cols
    out = empty(kind, rows, cols, device)
    out.copy_(torch.from_numpy(host[:, :cols]))
    return out


def to_host(t):
    """Copy a device matrix view to a contiguous numpy array (uint64 words
    for Boolean)."""
    import numpy as np
    a = t.detach().cpu().contiguous().numpy()
    if a.dtype == np.int64:
        a = a.view(np.uint64)
    return a


__all__ = [
    "SR_BOOL", "SR_ANTIDIST_U8", "SR_ANTIDIST_U16", "SR_DISTANCE_U8", "SR_DISTANCE_U16",
    "SR_ANTIDIST_U32", "SR_DISTANCE_U32", "elem_bytes",
    "SR_BOOL_M4R", "SR_CLOSURE_SQUARING", "SR_CLOSURE_WARSHALL", "SR_CLOSURE_BIG_BLOCKS",
    "autotune_closure", "autotune_mul", "autotune_clear", "SR_BATCH_TILE_AUTO",
    "SR_BATCH_TILE_64x16", "SR_BATCH_TILE_64x32", "SR_BATCH_TILE_64x64",
    "SR_EW_AND", "SR_EW_OR", "SR_EW_XOR", "SR_EW_NOT", "semiring_ewise", "SR_OK", "SR_EINVAL",
    "SR_EALIAS",
    "SR_EALIGN", "SR_ENOMEM", "SR_EDEVICE", "SR_EUNSUPPORTED", "SR_ACCUMULATE",
    "SR_REFLEXIVE", "SR_BOOL_BITWISE", "SR_BOOL_MFMA", "SR_SERIAL_PHASES", "SemiringError", "lib", "kind_of",
    "semiring_mul", "semiring_add", "closure", "closure_batched", "version", "shutdown",
    "sr_profile_enable", "sr_profile_read", "SR_PHASE_PIVOT", "SR_PHASE_PANELS",
    "SR_PHASE_UPDATE",
    "padded_ld", "empty", "clone", "to_device", "to_host", "BatchArena", "PreparedBatch",
    "EXPORTS", "LIB_PATH",
]
