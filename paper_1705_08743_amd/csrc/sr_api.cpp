// C-ABI front end of libsemiring (declared in include/semiring.h): argument
// validation on the host, dispatch to the HIP launchers, uint8 working copies,
// error reporting.  No torch types and no C++ exceptions cross this boundary.
#include <hip/hip_runtime_api.h>

#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <memory>
#include <mutex>
#include <numeric>
#include <set>
#include <string>
#include <vector>

#include "semiring.h"
#include "sr_internal.h"

namespace {

thread_local std::string g_err = "no error";

int vfail(int code, const char *fmt, va_list ap) {
    char buf[512];
    vsnprintf(buf, sizeof buf, fmt, ap);
    g_err = buf;
    return code;
}

int fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vfail(code, fmt, ap);
    va_end(ap);
    return code;
}

int ok() { return SR_OK; }

int device_fail(hipError_t e, const char *what) {
    return fail(SR_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

bool valid_kind(int kind) { return kind >= SR_BOOL && kind <= SR_DISTANCE_U32; }

bool is_dist(int kind) {
    return kind == SR_DISTANCE_U8 || kind == SR_DISTANCE_U16 || kind == SR_DISTANCE_U32;
}

// The anti-distance kind of the same width (distance kinds are computed as
// anti-distance ones through the De Morgan laws: not a = S - a).
int base_kind(int kind) {
    if (kind == SR_DISTANCE_U8) return SR_ANTIDIST_U8;
    if (kind == SR_DISTANCE_U16) return SR_ANTIDIST_U16;
    if (kind == SR_DISTANCE_U32) return SR_ANTIDIST_U32;
    return kind;
}

// Default size range of the repeated-squaring closure, from the measured
// crossover with the blocked loop on MI355X (uint16 / uint8: 2.4-4.6x faster
// for 256 <= D <= 1024, slower at D = 128 and from 1536 on; uint32: 10-25 %
// faster up to 768; Boolean: the blocked loop is faster at every size), and
// with big pivot blocks (uint16 / uint8, configuration-2 graphs: squaring
// 159 / 131 us at D = 640, big blocks 226 / 233; at 768 207 / 188 against
// 183 / 179, at 1024 321 / 290 against 217 / 209).
constexpr int64_t kSquaringMinD = 192;
// Boolean defaults for the matrix cores: products with every dimension at
// least kBoolMfmaMinDim, and the closure's bulk update from kBoolMfmaClosureD
// vertices on (configuration-3-like graphs: D = 2048 0.41 vs 0.43 ms, 8192
// 1.68 vs 1.83, 16384 4.49 vs 4.85 ms against the word kernels' best; equal
// at 1024).
constexpr int64_t kBoolMfmaMinDim = 512;
constexpr int64_t kBoolMfmaClosureD = 2048;
// Big-block closure (pivot blocks of kBigBlock closed by squaring) above the
// squaring range, up to these sizes (configuration-2-like graphs, us, against
// whole-matrix squaring and the 128-pivot loop: uint16 D = 768 149 / 185 /
// 428, 1024 183 / 288 / 567, 1536 331 / 1135 / 853, 2048 644 / - / 1129,
// 3072 1607 / - / 1766; uint8 alike; at 4096, where a round's products no
// longer share a launch, the loop wins (3.3 vs 4.3 ms); 512 the best block
// of 256 / 512 / 768 / 1024; uint32: 640 205 / 284 / 861, 768 276 / 239 /
// 1060, 1024 488 / 287 / 1385, 2048 - / 1012 / 3034, 3072 - / 2309 / 4545,
// 4096 - / 4509 / 6702).
constexpr int64_t kBigBlock = 512;
constexpr int64_t kBigBlockMaxD16 = 3072;
constexpr int64_t kBigBlockMaxD32 = 4096;
constexpr int64_t kSquaringMaxD16 = 704;
constexpr int64_t kSquaringMaxD32 = 704;

// bytes per storage unit of the leading dimension
int64_t unit_bytes(int kind) {
    switch (base_kind(kind)) {
        case SR_BOOL: return 8;
        case SR_ANTIDIST_U8: return 1;
        case SR_ANTIDIST_U16: return 2;
        default: return 4;
    }
}

// storage units needed per row for `cols` columns
int64_t row_units(int kind, int64_t cols) { return kind == SR_BOOL ? (cols + 63) / 64 : cols; }

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// Validates one matrix operand: rows x cols with leading dimension ld.
int check_matrix(int kind, const char *name, const void *p, int64_t ld, int64_t rows,
                 int64_t cols) {
    if (rows < 0 || cols < 0) return fail(SR_EINVAL, "%s: negative extent", name);
    if (ld < row_units(kind, cols))
        return fail(SR_EINVAL, "%s: ld=%lld is less than the row width (%lld %s)", name,
                    (long long)ld, (long long)row_units(kind, cols),
                    kind == SR_BOOL ? "64-bit words" : "elements");
    if (rows == 0 || cols == 0) return SR_OK;
    if (p == nullptr) return fail(SR_EINVAL, "%s: NULL pointer with nonzero extent", name);
    if (!aligned16(p)) return fail(SR_EALIGN, "%s: base pointer not 16-byte aligned", name);
    if ((ld * unit_bytes(kind)) % 16 != 0)
        return fail(SR_EALIGN, "%s: row stride of %lld bytes is not a multiple of 16", name,
                    (long long)(ld * unit_bytes(kind)));
    return SR_OK;
}

struct Span {
    uintptr_t lo, hi;  // [lo, hi)
};

Span span_of(int kind, const void *p, int64_t ld, int64_t rows) {
    const uintptr_t b = reinterpret_cast<uintptr_t>(p);
    return Span{b, b + (uintptr_t)(rows * ld * unit_bytes(kind))};
}

bool overlap(Span a, Span b) { return a.lo < b.hi && b.lo < a.hi; }

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

hipStream_t as_stream(void *s) { return static_cast<hipStream_t>(s); }

// Stream-ordered working memory for uint8 problems (widened to 16-bit
// working copies).
std::once_flag g_pool_once;

void configure_pool() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, dev) != hipSuccess) return;
    uint64_t threshold = UINT64_MAX;
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &threshold);
}

int work_alloc(void **p, size_t bytes, hipStream_t st) {
    std::call_once(g_pool_once, configure_pool);
    hipError_t e = hipMallocAsync(p, bytes, st);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(SR_ENOMEM, "could not allocate %zu bytes of working memory: %s", bytes,
                    hipGetErrorString(e));
    }
    return SR_OK;
}

void work_free(void *p, hipStream_t st) {
    if (p) (void)hipFreeAsync(p, st);
}

// The product after validation; kind is SR_BOOL or an anti-distance kind.
int mul_compute(int kind, void *C, int64_t ldc, const void *A, int64_t lda, const void *B,
                int64_t ldb, int64_t R, int64_t K, int64_t N, bool acc, unsigned path,
                hipStream_t st) {
    int rc;
    hipError_t e = hipSuccess;
    if (kind == SR_BOOL && path == SR_BOOL_MFMA) {
        void *w = nullptr;
        const size_t bytes = std::max<size_t>(sr::bool_mfma_work_bytes(R, K, N), 256);
        if ((rc = work_alloc(&w, bytes, st)) != SR_OK) return rc;
        e = sr::launch_bool_mul_mfma(static_cast<uint64_t *>(C), ldc,
                                     static_cast<const uint64_t *>(A), lda,
                                     static_cast<const uint64_t *>(B), ldb, R, K, N, acc, w, st);
        work_free(w, st);
    } else if (kind == SR_BOOL) {
        const int bp = path == SR_BOOL_M4R ? sr::kBoolPathM4r
                       : path == SR_BOOL_BITWISE ? sr::kBoolPathBitwise : sr::kBoolPathAuto;
        e = sr::launch_bool_mul(static_cast<uint64_t *>(C), ldc, static_cast<const uint64_t *>(A),
                                lda, static_cast<const uint64_t *>(B), ldb, R, K, N, acc, bp, st);
    } else if (kind == SR_ANTIDIST_U16) {
        e = sr::launch_ad_mul(false, static_cast<uint16_t *>(C), ldc,
                              static_cast<const uint16_t *>(A), lda,
                              static_cast<const uint16_t *>(B), ldb, R, K, N, acc, st);
    } else if (kind == SR_ANTIDIST_U32) {
        e = sr::launch_ad32_mul(static_cast<uint32_t *>(C), ldc, static_cast<const uint32_t *>(A),
                                lda, static_cast<const uint32_t *>(B), ldb, R, K, N, acc, st);
    } else {
        // uint8: widen to 16-bit working copies, multiply with S = 255, narrow.
        const int64_t lk = round_up(std::max<int64_t>(K, 1), 64);
        const int64_t ln = round_up(N, 64);
        const size_t bytes = (size_t)(R * lk + K * ln + R * ln) * 2;
        void *w = nullptr;
        if ((rc = work_alloc(&w, bytes, st)) != SR_OK) return rc;
        uint16_t *Aw = static_cast<uint16_t *>(w);
        uint16_t *Bw = Aw + R * lk;
        uint16_t *Cw = Bw + K * ln;
        const uint8_t *A8 = static_cast<const uint8_t *>(A);
        const uint8_t *B8 = static_cast<const uint8_t *>(B);
        uint8_t *C8 = static_cast<uint8_t *>(C);
        if (e == hipSuccess) e = sr::launch_widen_u8(Aw, lk, A8, lda, R, K, st);
        if (e == hipSuccess) e = sr::launch_widen_u8(Bw, ln, B8, ldb, K, N, st);
        if (e == hipSuccess && acc) e = sr::launch_widen_u8(Cw, ln, C8, ldc, R, N, st);
        if (e == hipSuccess) e = sr::launch_ad_mul(true, Cw, ln, Aw, lk, Bw, ln, R, K, N, acc, st);
        if (e == hipSuccess) e = sr::launch_narrow_u8(C8, ldc, Cw, ln, R, N, st);
        work_free(w, st);
    }
    if (e != hipSuccess) return device_fail(e, "semiring_mul launch");
    return ok();
}

}  // namespace

extern "C" {

const char *sr_last_error(void) { return g_err.c_str(); }

const char *sr_version(void) { return "libsemiring 0.1 (gfx950)"; }

int sr_profile_enable(int enable) { return sr::prof_enable(enable); }

int sr_profile_read(int kind, int phase, double *total_ms, int64_t *launches, double *updates) {
    if (!valid_kind(kind)) return fail(SR_EINVAL, "sr_profile_read: invalid kind %d", kind);
    if (phase < SR_PHASE_PIVOT || phase > SR_PHASE_UPDATE)
        return fail(SR_EINVAL, "sr_profile_read: invalid phase %d", phase);
    if (sr::prof_read(kind == SR_BOOL ? 0 : 1, phase, total_ms, launches, updates) != 0)
        return fail(SR_EDEVICE, "sr_profile_read: event query failed");
    return SR_OK;
}

void sr_shutdown(void) {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (int d = 0; d < n; d++) {
        if (hipSetDevice(d) != hipSuccess) continue;
        (void)hipDeviceSynchronize();
        hipMemPool_t pool;
        if (hipDeviceGetDefaultMemPool(&pool, d) == hipSuccess) (void)hipMemPoolTrimTo(pool, 0);
    }
    (void)hipSetDevice(cur);
}

int semiring_mul(int kind, void *C, int64_t ldc, const void *A, int64_t lda, const void *B,
                 int64_t ldb, int64_t R, int64_t K, int64_t N, unsigned flags, void *stream) {
    if (!valid_kind(kind)) return fail(SR_EINVAL, "semiring_mul: invalid kind %d", kind);
    const unsigned paths = flags & (SR_BOOL_BITWISE | SR_BOOL_MFMA | SR_BOOL_M4R);
    if (flags & ~(unsigned)(SR_ACCUMULATE | SR_BOOL_BITWISE | SR_BOOL_MFMA | SR_BOOL_M4R))
        return fail(SR_EINVAL, "semiring_mul: unknown flags 0x%x", flags);
    if (paths & (paths - 1))
        return fail(SR_EINVAL, "semiring_mul: at most one of SR_BOOL_BITWISE, SR_BOOL_MFMA, SR_BOOL_M4R");
    if ((flags & (SR_BOOL_MFMA | SR_BOOL_M4R)) && kind != SR_BOOL)
        return fail(SR_EINVAL, "semiring_mul: SR_BOOL_MFMA and SR_BOOL_M4R apply to SR_BOOL only");
    if (R < 0 || K < 0 || N < 0) return fail(SR_EINVAL, "semiring_mul: negative size");
    if (R > INT32_MAX || K > INT32_MAX || N > INT32_MAX)
        return fail(SR_EINVAL, "semiring_mul: sizes above 2^31-1 are not supported");
    int rc;
    if ((rc = check_matrix(kind, "C", C, ldc, R, N)) != SR_OK) return rc;
    if ((rc = check_matrix(kind, "A", A, lda, R, K)) != SR_OK) return rc;
    if ((rc = check_matrix(kind, "B", B, ldb, K, N)) != SR_OK) return rc;
    if (R == 0 || N == 0) return ok();
    const Span sc = span_of(kind, C, ldc, R);
    if (K > 0 && (overlap(sc, span_of(kind, A, lda, R)) || overlap(sc, span_of(kind, B, ldb, K))))
        return fail(SR_EALIAS,
                    "semiring_mul: C overlaps A or B (the in-place form is closure())");
    const bool acc = (flags & SR_ACCUMULATE) != 0;
    hipStream_t st = as_stream(stream);
    // Boolean without a forced path: the autotuned choice for this size
    // class, if any; else the matrix cores from 512 on in every dimension
    // (measured with 4-bit operands against the word kernels: 512^3 34 vs
    // 36 us, 4096^3 53 vs 197 us, 16384^3 1.92 vs 2.04 ms; 256^3 43 vs
    // 24 us); else the word kernels' own size rule
    unsigned path = paths;
    if (kind == SR_BOOL && !path) path = sr::tuned_get(sr::kTuneMul, kind, R, K, N);
    if (kind == SR_BOOL && !path && R >= kBoolMfmaMinDim && K >= kBoolMfmaMinDim &&
        N >= kBoolMfmaMinDim)
        path = SR_BOOL_MFMA;
    if (!is_dist(kind)) return mul_compute(kind, C, ldc, A, lda, B, ldb, R, K, N, acc, path, st);
    // distance product (min, saturating +) by De Morgan:
    // A + B = not((not A) (x) (not B)), with C complemented around it
    const int64_t es = unit_bytes(kind);
    const int64_t lk = round_up(std::max<int64_t>(K, 1), 64), ln = round_up(N, 64);
    void *w = nullptr;
    if ((rc = work_alloc(&w, (size_t)(R * lk + K * ln) * (size_t)es, st)) != SR_OK) return rc;
    char *nA = static_cast<char *>(w);
    char *nB = nA + R * lk * es;
    hipError_t e = sr::launch_ewise((int)es, sr::EW_NOT, nA, lk, A, lda, A, lda, R, K, 0, st);
    if (e == hipSuccess) e = sr::launch_ewise((int)es, sr::EW_NOT, nB, ln, B, ldb, B, ldb, K, N, 0, st);
    if (e == hipSuccess && acc)
        e = sr::launch_ewise((int)es, sr::EW_NOT, C, ldc, C, ldc, C, ldc, R, N, 0, st);
    if (e != hipSuccess) {
        work_free(w, st);
        return device_fail(e, "semiring_mul launch");
    }
    rc = mul_compute(base_kind(kind), C, ldc, nA, lk, nB, ln, R, K, N, acc, 0u, st);
    if (rc == SR_OK) {
        e = sr::launch_ewise((int)es, sr::EW_NOT, C, ldc, C, ldc, C, ldc, R, N, 0, st);
        if (e != hipSuccess) rc = device_fail(e, "semiring_mul launch");
    }
    work_free(w, st);
    return rc == SR_OK ? ok() : rc;
}

}  // extern "C"

namespace {

// Largest D for which closure() takes repeated squaring by default
// (SR_SQUARING_MAX_D overrides; 0 turns the default off).
int64_t squaring_max_d(int ak) {
    static const int64_t env = [] {
        const char *v = getenv("SR_SQUARING_MAX_D");
        return v ? (int64_t)atoll(v) : (int64_t)-1;
    }();
    if (env >= 0) return env;
    if (ak == SR_BOOL) return 0;
    return ak == SR_ANTIDIST_U32 ? kSquaringMaxD32 : kSquaringMaxD16;
}

bool capturing(hipStream_t st) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone;
}

// Pivot block of the big-block closure (SR_BIG_BLOCK overrides) and the
// largest D that takes it by default (SR_BIG_BLOCK_MAX_D overrides).
int64_t big_block_size() {
    static const int64_t b = [] {
        const char *v = getenv("SR_BIG_BLOCK");
        const int64_t x = v ? (int64_t)atoll(v) : kBigBlock;
        return x >= 128 ? round_up(x, 64) : kBigBlock;
    }();
    return b;
}
int64_t big_block_max_d(int ak) {
    static const int64_t env = [] {
        const char *v = getenv("SR_BIG_BLOCK_MAX_D");
        return v ? (int64_t)atoll(v) : (int64_t)-1;
    }();
    if (env >= 0) return env;
    return ak == SR_ANTIDIST_U32 ? kBigBlockMaxD32 : kBigBlockMaxD16;
}

// Closure by repeated squaring (eq. trcl: T = A * (I (+) A)^m for every
// m >= D - 1, because a best path never needs more than D - 1 edges before
// its last one): P := I (+) A, then j squarings P := P * P with 2^j >= D - 1,
// then T := A * P (for anti-distance entries without a product: P off the
// diagonal, the best cycle through each vertex on it).  Exact like every
// other path of the library; the products are the semiring_mul kernels.  For
// anti-distance entries the squarings stop on the device once one leaves P
// unchanged (below).  es: 2
// (uint16, or the binary16 form of uint8 data when s8), 4 (uint32), 8
// (Boolean words; ld in words).  work: squaring_work_bytes(es, D) bytes.
hipError_t closure_by_squaring(int es, bool s8, void *T, int64_t ld, int64_t D, void *work,
                               hipStream_t st) {
    const int64_t lw = es == 8 ? round_up((D + 63) / 64, 2) : round_up(D, 64);
    const int64_t row_bytes = es == 8 ? (D + 63) / 64 * 8 : D * es;
    char *P = static_cast<char *>(work);
    char *Q = P + D * lw * es;
    int j = 0;
    while ((int64_t(1) << j) < D - 1) j++;
    // I (+) A: the diagonal becomes the multiplicative one (S, or bit set)
    const uint32_t one = es == 4 ? 0xFFFFFFFFu : (es == 8 ? 1u : (s8 ? 0x5BF8u : 0xFFFFu));
    if (es == 8) {
        // Boolean rows must carry zero bits up to their padded end (the
        // product kernels read whole words there): P takes T's rows up to
        // lw <= ldt words, which are zero past D by the caller's contract, and
        // Q starts zeroed (the products write only the words that hold
        // columns < D).  Every squaring runs (the bit-sliced kernels take no
        // gate), then T := T * P.
        hipError_t e = hipMemcpy2DAsync(P, lw * es, T, ld * es, lw * 8, D,
                                        hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess)
            e = sr::launch_fill32(reinterpret_cast<uint32_t *>(Q), D * lw * 2, 0u, st);
        if (e == hipSuccess) e = sr::launch_diag(es, P, lw, D, one, st);
        auto mul = [&](void *C, const void *A, int64_t lda, const void *B) {
            return sr::launch_bool_mul(static_cast<uint64_t *>(C), lw,
                                       static_cast<const uint64_t *>(A), lda,
                                       static_cast<const uint64_t *>(B), lw, D, D, D, false,
                                       sr::kBoolPathAuto, st);
        };
        for (int i = 0; i < j && e == hipSuccess; i++) {
            e = mul(Q, P, lw, P);
            std::swap(P, Q);
        }
        if (e == hipSuccess) e = mul(Q, T, ld, P);
        if (e == hipSuccess)
            e = hipMemcpy2DAsync(T, ld * es, Q, lw * es, row_bytes, D, hipMemcpyDeviceToDevice,
                                 st);
        return e;
    }
    // Early exit on the device: squaring i compares each entry it stores
    // with P's and sets changed[i] if any differs; squaring i + 1 runs only if
    // that was set.  Once a squaring leaves P unchanged, P is idempotent and
    // every later power equals it; the skipped squarings leave both buffers
    // holding it.  The host enqueues all j squarings and never waits.
    int *changed = reinterpret_cast<int *>(static_cast<char *>(work) + 2 * D * lw * es);
    hipError_t e = sr::launch_power_prep(es, P, lw, T, ld, D, one, changed, j, st);
    for (int i = 0; i < j && e == hipSuccess; i++) {
        const int *gate = i == 0 ? nullptr : changed + i - 1;
        if (es == 4) {
            const uint32_t *p = reinterpret_cast<const uint32_t *>(P);
            e = sr::launch_ad32_mul(reinterpret_cast<uint32_t *>(Q), lw, p, lw, p, lw, D, D, D,
                                    false, st, -1, gate, p, changed + i);
        } else {
            const uint16_t *p = reinterpret_cast<const uint16_t *>(P);
            e = sr::launch_ad_mul(s8, reinterpret_cast<uint16_t *>(Q), lw, p, lw, p, lw, D, D, D,
                                  false, st, -1, gate, p, changed + i);
        }
        std::swap(P, Q);
    }
    // T := A * P without a product: P off the diagonal, the best cycle
    // through i on it (see launch_power_finish)
    if (e != hipSuccess) return e;
    return sr::launch_power_finish(es, s8, T, ld, P, lw, D, st);
}

// Blocked closure with large pivot blocks (Sec. II / Sec. III Warshall loop
// blocked by B pivots): per round K = [k0, k0 + bs), the pivot block is closed
// by repeated squaring, then the panels T_Kj (+)= T_KK * T_Kj and
// T_iK (+)= T_iK * T_KK, then T_ij (+)= T_iK * T_Kj, all as products on
// blocks of T.  A panel product's output block is also one of its operands;
// that is exact because T_KK is closed (T_KK * T_KK <= T_KK), so a mix of old
// and new operand entries gives the same result, as in the blocked kernels.
// For sizes where the 128-pivot loop's chain of pivot steps dominates but
// squaring the whole matrix would cost too many products.  es: 2 (uint16,
// or the binary16 form when s8) or 4 (uint32).  work: squaring_work_bytes of
// one block.
hipError_t closure_big_blocks(int es, bool s8, void *T, int64_t ld, int64_t D, int64_t B,
                              void *work, hipStream_t st) {
    char *base = static_cast<char *>(T);
    auto at = [&](int64_t r, int64_t c) { return base + (r * ld + c) * es; };
    // C (+)= A * B on blocks of T (B's rows end at column D of T); the up to
    // four panel products of a round share one launch, and so do the up to
    // four block products (they are independent: every panel product writes
    // its own panel, and the block products read only the finished panels)
    sr::MulDesc group[4];
    sr::MulDesc32 group32[4];
    int ng = 0;
    auto add = [&](int64_t cr, int64_t cc, int64_t ar, int64_t ac, int64_t br, int64_t bc,
                   int64_t R, int64_t K, int64_t N) -> hipError_t {
        if (R <= 0 || K <= 0 || N <= 0) return hipSuccess;
        if (es == 4)
            group32[ng++] = {reinterpret_cast<uint32_t *>(at(cr, cc)),
                             reinterpret_cast<const uint32_t *>(at(ar, ac)),
                             reinterpret_cast<const uint32_t *>(at(br, bc)), ld, ld, ld, R, K, N,
                             ld - bc};
        else
            group[ng++] = {reinterpret_cast<uint16_t *>(at(cr, cc)),
                           reinterpret_cast<const uint16_t *>(at(ar, ac)),
                           reinterpret_cast<const uint16_t *>(at(br, bc)), ld, ld, ld, R, K, N,
                           ld - bc};
        return hipSuccess;
    };
    auto flush = [&]() -> hipError_t {
        if (ng == 0) return hipSuccess;
        hipError_t e = es == 4 ? sr::launch_ad32_mul_group(group32, ng, true, st)
                               : sr::launch_ad_mul_group(s8, group, ng, true, st);
        ng = 0;
        return e;
    };
    hipError_t e = hipSuccess;
    for (int64_t k0 = 0; k0 < D && e == hipSuccess; k0 += B) {
        const int64_t bs = std::min(B, D - k0), k1 = k0 + bs;
        e = closure_by_squaring(es, s8, at(k0, k0), ld, bs, work, st);
        // row panel (left, right of the pivot block), column panel (above, below)
        if (e == hipSuccess) e = add(k0, 0, k0, k0, k0, 0, bs, bs, k0);
        if (e == hipSuccess) e = add(k0, k1, k0, k0, k0, k1, bs, bs, D - k1);
        if (e == hipSuccess) e = add(0, k0, 0, k0, k0, k0, k0, bs, bs);
        if (e == hipSuccess) e = add(k1, k0, k1, k0, k0, k0, D - k1, bs, bs);
        if (e == hipSuccess) e = flush();
        // the four blocks outside the pivot rows and columns
        const int64_t rows[2][2] = {{0, k0}, {k1, D - k1}};
        for (const auto &r : rows)
            for (const auto &c : rows)
                if (e == hipSuccess) e = add(r[0], c[0], r[0], k0, k0, c[0], r[1], bs, c[1]);
        if (e == hipSuccess) e = flush();
    }
    return e;
}

size_t squaring_work_bytes(int es, int64_t D) {
    const int64_t lw = es == 8 ? round_up((D + 63) / 64, 2) : round_up(D, 64);
    return (size_t)(2 * D * lw * es) + 256;  // P, Q, then the changed[] flags (j <= 64)
}

// Validation shared by semiring_add and semiring_ewise (B unused for NOT).
int ewise_checked(const char *fn, int kind, int op, void *C, int64_t ldc, const void *A,
                  int64_t lda, const void *B, int64_t ldb, int64_t R, int64_t N, void *stream) {
    if (!valid_kind(kind)) return fail(SR_EINVAL, "%s: invalid kind %d", fn, kind);
    if (op < sr::EW_AND || op > sr::EW_NOT) return fail(SR_EINVAL, "%s: invalid op %d", fn, op);
    if (R < 0 || N < 0) return fail(SR_EINVAL, "%s: negative size", fn);
    const bool unary = op == sr::EW_NOT;
    int rc;
    if ((rc = check_matrix(kind, "C", C, ldc, R, N)) != SR_OK) return rc;
    if ((rc = check_matrix(kind, "A", A, lda, R, N)) != SR_OK) return rc;
    if (!unary && (rc = check_matrix(kind, "B", B, ldb, R, N)) != SR_OK) return rc;
    if (R == 0 || N == 0) return ok();
    const Span sc = span_of(kind, C, ldc, R);
    const bool same_a = (C == A && ldc == lda), same_b = (C == B && ldc == ldb);
    if ((!same_a && overlap(sc, span_of(kind, A, lda, R))) ||
        (!unary && !same_b && overlap(sc, span_of(kind, B, ldb, R))))
        return fail(SR_EALIAS, "%s: C partially overlaps A or B", fn);
    const int64_t units = row_units(kind, N);
    hipError_t e = sr::launch_ewise((int)unit_bytes(kind), op, C, ldc, A, lda, unary ? A : B,
                                    unary ? lda : ldb, R, units, N, as_stream(stream));
    if (e != hipSuccess) return device_fail(e, "entrywise launch");
    return ok();
}

}  // namespace

namespace {

// Working memory of a closure by method m: the binary16 copy of uint8 data,
// then the two matrices of squaring (of the whole matrix, or of one big
// block), or the transposed pivot rows of the Boolean matrix-core update.
size_t closure_need(int kind, int64_t D, unsigned m, unsigned bool_path, int64_t block) {
    const int ak = base_kind(kind);
    const bool s8 = ak == SR_ANTIDIST_U8;
    const size_t tw = s8 ? (size_t)(D * round_up(D, 64)) * 2 : 0;
    if (m == SR_CLOSURE_WARSHALL)
        return ak == SR_BOOL && (bool_path & SR_BOOL_MFMA) ? sr::bool_mfma_closure_work_bytes(D)
                                                           : tw;
    const int wes = s8 ? 2 : (int)unit_bytes(kind);
    const int64_t b = m == SR_CLOSURE_BIG_BLOCKS ? std::min<int64_t>(block, D) : D;
    return tw + squaring_work_bytes(wes, b);
}

// An autotuned closure choice holds the method flags and, for big pivot
// blocks, the block size in units of 64 vertices in bits 16..23 (0: the
// default size).
constexpr unsigned kTunedBlockShift = 16;
constexpr unsigned kTunedMethodMask = 0xFFFFu;
unsigned tuned_block_code(int64_t block) { return (unsigned)(block / 64) << kTunedBlockShift; }
int64_t tuned_block(unsigned choice) {
    const int64_t b = (int64_t)((choice >> kTunedBlockShift) & 0xFFu) * 64;
    return b > 0 ? b : big_block_size();
}

// Kind, size and flags of a closure call (the matrix is checked apart).
int check_closure_args(int kind, int64_t D, unsigned flags, const char *fn) {
    if (!valid_kind(kind)) return fail(SR_EINVAL, "%s: invalid kind %d", fn, kind);
    const unsigned methods = flags & (SR_CLOSURE_SQUARING | SR_CLOSURE_WARSHALL |
                                      SR_CLOSURE_BIG_BLOCKS);
    if (flags & ~(unsigned)(SR_REFLEXIVE | SR_BOOL_BITWISE | SR_BOOL_MFMA | SR_BOOL_M4R |
                            SR_SERIAL_PHASES | SR_CLOSURE_SQUARING | SR_CLOSURE_WARSHALL |
                            SR_CLOSURE_BIG_BLOCKS))
        return fail(SR_EINVAL, "%s: unknown flags 0x%x", fn, flags);
    const unsigned paths = flags & (SR_BOOL_BITWISE | SR_BOOL_M4R | SR_BOOL_MFMA);
    if (paths & (paths - 1))
        return fail(SR_EINVAL, "%s: at most one of SR_BOOL_BITWISE, SR_BOOL_M4R, SR_BOOL_MFMA", fn);
    if ((flags & SR_BOOL_MFMA) && base_kind(kind) != SR_BOOL)
        return fail(SR_EINVAL, "%s: SR_BOOL_MFMA applies to SR_BOOL only", fn);
    if (methods & (methods - 1))
        return fail(SR_EINVAL, "%s: at most one of SR_CLOSURE_SQUARING, "
                               "SR_CLOSURE_WARSHALL, SR_CLOSURE_BIG_BLOCKS", fn);
    if ((flags & SR_CLOSURE_BIG_BLOCKS) && base_kind(kind) == SR_BOOL)
        return fail(SR_EUNSUPPORTED, "%s: SR_CLOSURE_BIG_BLOCKS is for non-Boolean kinds", fn);
    if (D < 0) return fail(SR_EINVAL, "%s: negative size", fn);
    if (D > INT32_MAX) return fail(SR_EINVAL, "%s: sizes above 2^31-1 are not supported", fn);
    return SR_OK;
}

struct ClosurePlan {
    unsigned method, bool_path;
    int64_t block;  // pivot block of the big-block method
    size_t copy_bytes, work_bytes;
};

// The method: forced by a flag; else the autotuned choice for this size
// class, if any; else the built-in size rules -- repeated squaring for small
// anti-distance matrices (where the blocked loop's chain of D sequential
// pivot steps dominates), big pivot blocks closed by squaring for mid sizes,
// the blocked loop otherwise; loop_only (a capture without caller-supplied
// working memory) turns a default squaring or big-block choice into the loop.
// Flags are valid (checked by the caller).
ClosurePlan plan_closure(int kind, int64_t D, unsigned flags, bool loop_only,
                         int64_t block = 0) {
    const int ak = base_kind(kind);
    unsigned method = flags & (SR_CLOSURE_SQUARING | SR_CLOSURE_WARSHALL | SR_CLOSURE_BIG_BLOCKS);
    unsigned bool_path = flags & (SR_BOOL_BITWISE | SR_BOOL_M4R | SR_BOOL_MFMA);
    int64_t big = block > 0 ? block : big_block_size();
    if (!method && (flags & SR_SERIAL_PHASES)) method = SR_CLOSURE_WARSHALL;
    if (!method) {
        const unsigned t = sr::tuned_get(sr::kTuneClosure, kind, D, 0, 0);
        if (t) {
            if (block <= 0) big = tuned_block(t);
            method = t & (SR_CLOSURE_SQUARING | SR_CLOSURE_WARSHALL | SR_CLOSURE_BIG_BLOCKS);
            if (!bool_path) bool_path = t & (SR_BOOL_BITWISE | SR_BOOL_M4R | SR_BOOL_MFMA);
        } else if (D >= kSquaringMinD && D <= squaring_max_d(ak)) {
            method = SR_CLOSURE_SQUARING;
        } else if (ak != SR_BOOL && D > squaring_max_d(ak) && D <= big_block_max_d(ak)) {
            method = SR_CLOSURE_BIG_BLOCKS;
        } else {
            method = SR_CLOSURE_WARSHALL;
        }
        if (method != SR_CLOSURE_WARSHALL && loop_only) method = SR_CLOSURE_WARSHALL;
    }
    // the Boolean loop's bulk update: the matrix cores by default for large
    // matrices, unless the stream is being captured without caller-supplied
    // working memory (their transposed pivot rows need some)
    if (ak == SR_BOOL && !bool_path && method == SR_CLOSURE_WARSHALL && D >= kBoolMfmaClosureD &&
        !loop_only)
        bool_path = SR_BOOL_MFMA;
    ClosurePlan p;
    p.method = method;
    p.bool_path = bool_path;
    p.block = big;
    p.copy_bytes = ak == SR_ANTIDIST_U8 ? (size_t)(D * round_up(D, 64)) * 2 : 0;
    p.work_bytes = closure_need(kind, D, method, bool_path, big);
    return p;
}

}  // namespace

namespace sr {

int closure_run(int kind, void *T, int64_t ldt, int64_t D, unsigned flags, void *stream,
                int (*fixed_work)(void **), size_t fixed_bytes, const char *fn, int64_t block) {
    const bool fixed = fixed_work != nullptr;
    int rc = check_closure_args(kind, D, flags, fn);
    if (rc != SR_OK) return rc;
    const unsigned methods = flags & (SR_CLOSURE_SQUARING | SR_CLOSURE_WARSHALL |
                                      SR_CLOSURE_BIG_BLOCKS);
    const bool serial = (flags & SR_SERIAL_PHASES) != 0;
    if ((rc = check_matrix(kind, "T", T, ldt, D, D)) != SR_OK) return rc;
    if (D == 0) return ok();
    hipStream_t st = as_stream(stream);
    hipError_t e = hipSuccess;
    const int es = (int)unit_bytes(kind);
    const int ak = base_kind(kind);
    // The method, the Boolean bulk-update path and the working memory.  A
    // stream being captured takes the loop unless the caller supplied the
    // working memory.
    ClosurePlan pl = plan_closure(kind, D, flags, !fixed && capturing(st), block);
    unsigned method = pl.method;
    const unsigned bool_path = pl.bool_path;
    const bool s8 = ak == SR_ANTIDIST_U8;
    const int64_t lw = round_up(D, 64);
    const size_t tw = pl.copy_bytes;
    const int wes = s8 ? 2 : es;
    const bool bool_mfma = ak == SR_BOOL && (bool_path & SR_BOOL_MFMA);
    size_t need = pl.work_bytes;
    void *w = nullptr;
    if (fixed) {
        // the caller's buffer: a method chosen by default that needs more
        // falls back to the loop, which needs only the uint8 working copy
        if (need > fixed_bytes && !methods && method != SR_CLOSURE_WARSHALL) {
            method = SR_CLOSURE_WARSHALL;
            need = closure_need(kind, D, method, bool_path, pl.block);
        }
        if (need > fixed_bytes)
            return fail(SR_EINVAL,
                        "%s: D=%lld needs %zu bytes of working memory, more than the %zu bytes "
                        "of the static scratch",
                        fn, (long long)D, need, fixed_bytes);
        if (need > 0 && (rc = fixed_work(&w)) != SR_OK) return rc;
    } else if (need > 0 && (rc = work_alloc(&w, std::max<size_t>(need, 256), st)) != SR_OK) {
        return rc;
    }
    const bool big = method == SR_CLOSURE_BIG_BLOCKS;
    const bool squared = method != SR_CLOSURE_WARSHALL;
    const int64_t B = big ? std::min<int64_t>(pl.block, D) : D;
    const bool aux_create = !fixed;
    // distance closure (dransclose) by De Morgan: not closure(not T)
    if (is_dist(kind)) e = sr::launch_ewise(es, sr::EW_NOT, T, ldt, T, ldt, T, ldt, D, D, 0, st);
    // the matrix the method runs on: T, or the binary16 copy of uint8 data
    void *M = T;
    int64_t ldm = ldt;
    if (e == hipSuccess && s8) {
        M = w;
        ldm = lw;
        e = sr::launch_widen_u8(static_cast<uint16_t *>(M), lw, static_cast<uint8_t *>(T), ldt, D,
                                D, st);
    }
    if (e == hipSuccess && squared) {
        void *work = static_cast<char *>(w) + tw;
        e = big ? closure_big_blocks(wes, s8, M, ldm, D, B, work, st)
                : closure_by_squaring(wes, s8, M, ldm, D, work, st);
    } else if (e == hipSuccess && ak == SR_BOOL) {
        const int path = (bool_path & SR_BOOL_M4R)       ? sr::kBoolPathM4r
                         : (bool_path & SR_BOOL_BITWISE) ? sr::kBoolPathBitwise
                         : bool_mfma                     ? sr::kBoolPathMfma
                                                         : sr::kBoolPathAuto;
        e = sr::launch_bool_closure(static_cast<uint64_t *>(T), ldt, D, serial, path, st,
                                     aux_create, w);
    } else if (e == hipSuccess && ak == SR_ANTIDIST_U32) {
        e = sr::launch_ad32_closure(static_cast<uint32_t *>(T), ldt, D, serial, st, aux_create);
    } else if (e == hipSuccess) {
        e = sr::launch_ad_closure(s8, static_cast<uint16_t *>(M), ldm, D, serial, st,
                                   aux_create);
    }
    if (e == hipSuccess && s8)
        e = sr::launch_narrow_u8(static_cast<uint8_t *>(T), ldt, static_cast<uint16_t *>(M), lw, D,
                                 D, st);
    if (!fixed) work_free(w, st);
    if (e == hipSuccess && is_dist(kind))
        e = sr::launch_ewise(es, sr::EW_NOT, T, ldt, T, ldt, T, ldt, D, D, 0, st);
    // reflexive closure I (+) T (eq. rtc): the diagonal of the multiplicative
    // identity -- S (anti-distance), 0 (distance), 1 (Boolean)
    if (e == hipSuccess && (flags & SR_REFLEXIVE)) {
        const uint32_t one = is_dist(kind) ? 0u
                             : kind == SR_ANTIDIST_U8  ? 255u
                             : kind == SR_ANTIDIST_U16 ? 65535u
                                                       : 0xFFFFFFFFu;
        e = sr::launch_diag(es, T, ldt, D, one, st);
    }
    if (e != hipSuccess) return fail(SR_EDEVICE, "%s launch: %s", fn, hipGetErrorString(e));
    return ok();
}

int report(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vfail(code, fmt, ap);
    va_end(ap);
    return code;
}

}  // namespace sr

extern "C" {

int semiring_add(int kind, void *C, int64_t ldc, const void *A, int64_t lda, const void *B,
                 int64_t ldb, int64_t R, int64_t N, void *stream) {
    // (+) is max for anti-distance and Boolean entries, min for distances
    return ewise_checked("semiring_add", kind, is_dist(kind) ? sr::EW_AND : sr::EW_OR, C, ldc, A,
                         lda, B, ldb, R, N, stream);
}

int semiring_ewise(int kind, int op, void *C, int64_t ldc, const void *A, int64_t lda,
                   const void *B, int64_t ldb, int64_t R, int64_t N, void *stream) {
    return ewise_checked("semiring_ewise", kind, op, C, ldc, A, lda, B, ldb, R, N, stream);
}

int closure(int kind, void *T, int64_t ldt, int64_t D, unsigned flags, void *stream) {
    return sr::closure_run(kind, T, ldt, D, flags, stream, nullptr, 0, "closure");
}

int64_t closure_work_bytes(int kind, int64_t D, unsigned flags) {
    const int rc = check_closure_args(kind, D, flags, "closure_work_bytes");
    if (rc != SR_OK) return rc;
    if (D == 0) return 0;
    const size_t need = plan_closure(kind, D, flags, false).work_bytes;
    return need > 0 ? (int64_t)std::max<size_t>(need, 256) : 0;
}

}  // extern "C"

namespace {

// Validates a batch as closure_batched documents (fn names the entry point
// in the messages).
int check_batch(const char *fn, int kind, void *const *T, const int64_t *ldt, const int64_t *D,
                int64_t count, unsigned flags) {
    if (!valid_kind(kind)) return fail(SR_EINVAL, "%s: invalid kind %d", fn, kind);
    if (flags & ~(unsigned)SR_REFLEXIVE) return fail(SR_EINVAL, "%s: unknown flags 0x%x", fn, flags);
    if (count < 0) return fail(SR_EINVAL, "%s: negative count", fn);
    if (count == 0) return ok();
    if (count > INT32_MAX) return fail(SR_EINVAL, "%s: count above 2^31-1", fn);
    if (!T || !ldt || !D) return fail(SR_EINVAL, "%s: NULL descriptor array", fn);
    std::vector<Span> spans;
    spans.reserve((size_t)count);
    for (int64_t g = 0; g < count; g++) {
        if (D[g] > 65536) return fail(SR_EINVAL, "%s: D[%lld] too large", fn, (long long)g);
        if (check_matrix(kind, "T[g]", T[g], ldt[g], D[g], D[g]) != SR_OK) {
            char name[48];  // formatted only on failure: the check again, naming g
            snprintf(name, sizeof name, "%s: T[%lld]", fn, (long long)g);
            return check_matrix(kind, name, T[g], ldt[g], D[g], D[g]);
        }
        if (D[g] > 0) spans.push_back(span_of(kind, T[g], ldt[g], D[g]));
    }
    std::sort(spans.begin(), spans.end(), [](Span a, Span b) { return a.lo < b.lo; });
    for (size_t i = 1; i < spans.size(); i++)
        if (spans[i].lo < spans[i - 1].hi)
            return fail(SR_EALIAS, "%s: two matrices of the batch overlap", fn);
    return ok();
}

// Batches computed in a 16-bit working copy (binary16 values): uint8 data,
// and Boolean data as {0, 255} anti-distance matrices.
bool batch_in_copies(int kind) { return kind == SR_BOOL || base_kind(kind) == SR_ANTIDIST_U8; }

// The batch's descriptors, largest graph first (ties keep the caller's
// order).  uint8 and Boolean kinds: T8 is the caller's matrix (ld8 in bytes)
// and T, the 16-bit working copy, is left null for place_working_copies;
// *work_elems receives the elements those copies take.
std::vector<sr::BatchDesc> batch_descs(int kind, void *const *T, const int64_t *ldt,
                                       const int64_t *D, int64_t count, size_t *work_elems) {
    const bool s8 = batch_in_copies(kind);
    std::vector<int64_t> order((size_t)count);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return D[a] > D[b]; });
    std::vector<sr::BatchDesc> h((size_t)count);
    *work_elems = 0;
    for (int64_t i = 0; i < count; i++) {
        const int64_t g = order[(size_t)i];
        sr::BatchDesc &d = h[(size_t)i];
        d.D = (int32_t)D[g];
        d.flags = 0;
        d.T32 = nullptr;
        if (s8) {
            d.T8 = static_cast<uint8_t *>(T[g]);
            d.ld8 = ldt[g] * unit_bytes(kind);
            d.ld = round_up(D[g], 8);
            d.T = nullptr;
            if (kind == SR_BOOL && D[g] <= sr::kBoolBatchSmall)
                d.flags = sr::kDescBits;  // closed on its bits: no working copy
            else
                *work_elems += (size_t)(D[g] * d.ld);
        } else if (base_kind(kind) == SR_ANTIDIST_U32) {
            d.T8 = nullptr;
            d.ld8 = 0;
            d.T = nullptr;
            d.T32 = static_cast<uint32_t *>(T[g]);
            d.ld = ldt[g];
        } else {
            d.T8 = nullptr;
            d.ld8 = 0;
            d.T = static_cast<uint16_t *>(T[g]);
            d.ld = ldt[g];
        }
    }
    return h;
}

// Points the uint8 descriptors' working copies at consecutive pieces of
// `arena` (16-bit elements; the pieces are multiples of 16 bytes).
void place_working_copies(std::vector<sr::BatchDesc> &h, void *arena) {
    uint16_t *a = static_cast<uint16_t *>(arena);
    size_t off = 0;
    for (sr::BatchDesc &d : h) {
        if (d.flags & sr::kDescBits) continue;
        d.T = a + off;
        off += (size_t)d.D * (size_t)d.ld;
    }
}

constexpr const char *kPlanFailure =
    "could not build the batch's work lists (a launch would number more than 2^31 - 4 "
    "workgroups, or host memory ran out)";

int closure_batched_impl(int kind, void *const *T, const int64_t *ldt, const int64_t *D,
                         int64_t count, unsigned flags, void *stream);

// Update-tile shape for a batch: SR_BATCH_TILE (1, 2, 3) if set, else the
// autotuned choice for its class, else the default.
bool batch_wide(int kind) { return base_kind(kind) == SR_ANTIDIST_U32; }

int batch_tile_for(int kind, const std::vector<sr::BatchDesc> &h) {
    if (batch_wide(kind)) return SR_BATCH_TILE_64x32;  // the one 32-bit shape
    static const int forced = [] {
        const char *v = getenv("SR_BATCH_TILE");
        const int t = v ? atoi(v) : 0;
        return t >= 1 && t <= 3 ? t : 0;
    }();
    if (forced) return forced;
    const int64_t max_d = h.empty() ? 0 : h.front().D;
    const unsigned t = sr::tuned_get(sr::kTuneBatch, kind, max_d, (int64_t)h.size(), 0);
    return t ? (int)t : sr::kBatchTileDefault;
}

}  // namespace

extern "C" {

int closure_batched(int kind, void *const *T, const int64_t *ldt, const int64_t *D, int64_t count,
                    unsigned flags, void *stream) {
    try {
        return closure_batched_impl(kind, T, ldt, D, count, flags, stream);
    } catch (const std::bad_alloc &) {
        return fail(SR_ENOMEM, "closure_batched: out of host memory");
    }
}

}  // extern "C"

namespace {

int closure_batched_impl(int kind, void *const *T, const int64_t *ldt, const int64_t *D,
                         int64_t count, unsigned flags, void *stream) {
    int rc = check_batch("closure_batched", kind, T, ldt, D, count, flags);
    if (rc != SR_OK || count == 0) return rc;
    hipStream_t st = as_stream(stream);
    const bool s8 = batch_in_copies(kind);
    size_t work_elems = 0;
    std::vector<sr::BatchDesc> h = batch_descs(kind, T, ldt, D, count, &work_elems);
    // descriptors and per-round work lists, then the 16-bit working copies
    std::unique_ptr<sr::BatchPlan, void (*)(sr::BatchPlan *)> plan(
        sr::batch_plan_create(h.data(), count, batch_tile_for(kind, h)), sr::batch_plan_destroy);
    if (!plan) return fail(SR_EINVAL, "closure_batched: %s", kPlanFailure);
    const size_t plan_bytes = round_up((int64_t)sr::batch_plan_bytes(plan.get(), count), 256);
    void *w = nullptr;
    rc = work_alloc(&w, plan_bytes + work_elems * 2, st);
    if (rc != SR_OK) return rc;
    if (s8) place_working_copies(h, static_cast<char *>(w) + plan_bytes);
    hipError_t e = sr::launch_ad_closure_batched(s8, plan.get(), h.data(), count, w, is_dist(kind),
                                                 (flags & SR_REFLEXIVE) != 0, kind == SR_BOOL,
                                                 batch_wide(kind), st);
    work_free(w, st);
    if (e != hipSuccess) return device_fail(e, "closure_batched launch");
    return ok();
}

}  // namespace


namespace {

// Times `run` (which enqueues one call on st and returns an SR_* code) once
// to warm up and `reps` more times with hipEvents on st; returns the fastest
// in milliseconds, or a negative value when a run fails (an allocation, say).
template <class Run, class Reset>
float time_candidate(hipStream_t st, hipEvent_t e0, hipEvent_t e1, int reps, Reset reset, Run run) {
    float best = -1.0f;
    for (int i = 0; i <= reps; i++) {
        if (reset() != hipSuccess) return -1.0f;
        if (hipEventRecord(e0, st) != hipSuccess) return -1.0f;
        if (run() != SR_OK) return -1.0f;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
            return -1.0f;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return -1.0f;
        if (i > 0 && (best < 0.0f || ms < best)) best = ms;
    }
    return best;
}

struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    bool ok() {
        return hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess;
    }
    ~EventPair() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

}  // namespace

extern "C" {

int sr_autotune_closure(int kind, int64_t D, unsigned *chosen, void *stream) {
    if (!valid_kind(kind)) return fail(SR_EINVAL, "sr_autotune_closure: invalid kind %d", kind);
    if (D < 1 || D > 32768)
        return fail(SR_EINVAL, "sr_autotune_closure: D = %lld outside [1, 32768]", (long long)D);
    hipStream_t st = as_stream(stream);
    if (capturing(st))
        return fail(SR_EUNSUPPORTED, "sr_autotune_closure: the stream is being captured");
    const int ak = base_kind(kind);
    // The loop's and the big blocks' runtimes do not depend on the entries;
    // the squaring stops once a squaring changes nothing (except for
    // Boolean), so every candidate runs on the worst case for that stop: a
    // directed path 0 -> 1 -> ... -> D-1 of distance-1 edges, whose best
    // paths use all D - 1 edges (a Boolean matrix stays zero).
    const int64_t ld = ak == SR_BOOL ? round_up((D + 63) / 64, 2) : round_up(D, 64);
    const size_t bytes = (size_t)(D * ld * unit_bytes(kind));
    std::vector<unsigned> cands;
    if (ak == SR_BOOL) {
        cands = {SR_CLOSURE_WARSHALL | SR_BOOL_BITWISE, SR_CLOSURE_WARSHALL | SR_BOOL_M4R,
                 SR_CLOSURE_WARSHALL | SR_BOOL_MFMA};
    } else {
        cands = {SR_CLOSURE_WARSHALL};
        // big pivot blocks of 256 to 1024 vertices (the tuned choice carries
        // the block size)
        if (D <= 16384)
            for (int64_t B : {256, 512, 768, 1024})
                if (B < D) cands.push_back(SR_CLOSURE_BIG_BLOCKS | tuned_block_code(B));
    }
    if (D >= 2 && D <= 4096) cands.push_back(SR_CLOSURE_SQUARING);
    EventPair ev;
    if (!ev.ok()) return device_fail(hipErrorOutOfMemory, "sr_autotune_closure: events");
    void *T = nullptr;
    int rc = work_alloc(&T, bytes, st);
    if (rc != SR_OK) return rc;
    unsigned pick = 0;
    float best = 0.0f;
    const int es = (int)unit_bytes(kind);
    const uint32_t edge = is_dist(kind) ? 1u : (es == 1 ? 254u : (es == 2 ? 65534u : 0xFFFFFFFEu));
    auto path = [&]() -> hipError_t {
        // absent edges: 0 (anti-distance, Boolean) or S, all bits set (distance)
        hipError_t e = hipMemsetAsync(T, is_dist(kind) ? 0xFF : 0, bytes, st);
        if (e == hipSuccess && ak != SR_BOOL && D > 1)
            e = sr::launch_diag(es, static_cast<char *>(T) + es, ld, D - 1, edge, st);
        return e;
    };
    for (unsigned c : cands) {
        const float ms = time_candidate(st, ev.a, ev.b, 2, path, [&] {
            return sr::closure_run(kind, T, ld, D, c & kTunedMethodMask, stream, nullptr, 0,
                                   "sr_autotune_closure", tuned_block(c));
        });
        if (ms >= 0.0f && (!pick || ms < best)) {
            pick = c;
            best = ms;
        }
    }
    work_free(T, st);
    (void)hipStreamSynchronize(st);
    if (!pick) return fail(SR_EDEVICE, "sr_autotune_closure: no candidate ran");
    sr::tuned_set(sr::kTuneClosure, kind, D, 0, 0, pick);
    if (chosen) *chosen = pick & kTunedMethodMask;
    return ok();
}

int sr_autotune_mul(int kind, int64_t R, int64_t K, int64_t N, unsigned *chosen, void *stream) {
    if (kind != SR_BOOL)
        return fail(SR_EUNSUPPORTED, "sr_autotune_mul: only the Boolean product has several paths");
    if (R < 1 || K < 1 || N < 1 || R > 65536 || K > 65536 || N > 65536)
        return fail(SR_EINVAL, "sr_autotune_mul: sizes outside [1, 65536]");
    hipStream_t st = as_stream(stream);
    if (capturing(st))
        return fail(SR_EUNSUPPORTED, "sr_autotune_mul: the stream is being captured");
    const int64_t lk = round_up((K + 63) / 64, 2), ln = round_up((N + 63) / 64, 2);
    const size_t ba = (size_t)(R * lk * 8), bb = (size_t)(K * ln * 8), bc = (size_t)(R * ln * 8);
    EventPair ev;
    if (!ev.ok()) return device_fail(hipErrorOutOfMemory, "sr_autotune_mul: events");
    void *w = nullptr;
    int rc = work_alloc(&w, ba + bb + bc, st);
    if (rc != SR_OK) return rc;
    char *A = static_cast<char *>(w), *B = A + ba, *C = B + bb;
    unsigned pick = 0;
    float best = 0.0f;
    for (unsigned c : {SR_BOOL_BITWISE, SR_BOOL_M4R, SR_BOOL_MFMA}) {
        const float ms = time_candidate(
            st, ev.a, ev.b, 2, [&] { return hipMemsetAsync(w, 0, ba + bb + bc, st); },
            [&] { return semiring_mul(kind, C, ln, A, lk, B, ln, R, K, N, c, stream); });
        if (ms >= 0.0f && (!pick || ms < best)) {
            pick = c;
            best = ms;
        }
    }
    work_free(w, st);
    (void)hipStreamSynchronize(st);
    if (!pick) return fail(SR_EDEVICE, "sr_autotune_mul: no candidate ran");
    sr::tuned_set(sr::kTuneMul, kind, R, K, N, pick);
    if (chosen) *chosen = pick;
    return ok();
}

void sr_autotune_clear(void) { sr::tuned_clear(); }

int sr_autotune_save(const char *path) {
    if (!path) return fail(SR_EINVAL, "sr_autotune_save: NULL path");
    if (sr::tuned_save(path) != 0)
        return fail(SR_EINVAL, "sr_autotune_save: could not write %s", path);
    return ok();
}

int sr_autotune_load(const char *path) {
    if (!path) return fail(SR_EINVAL, "sr_autotune_load: NULL path");
    const int n = sr::tuned_load(path);
    if (n < 0) return fail(SR_EINVAL, "sr_autotune_load: could not read %s", path);
    return ok();
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Prepared batches

struct sr_batch {
    int kind = 0;
    int device = 0;
    bool s8 = false, dual = false, reflexive = false, bits = false, wide = false;
    int64_t count = 0;
    std::vector<sr::BatchDesc> h;  // largest first; uint8: working copies placed
    sr::BatchPlan *plan = nullptr;
    char *dev = nullptr;      // hipMalloc: the first plan image (image_cap bytes),
    size_t image_cap = 0;     // then the uint8 / Boolean working copies
    size_t work_elems = 0;
    char *image = nullptr;    // the current plan's device image (dev, or one of retired)
    // images of later plans (sr_batch_autotune): each re-plan uploads into a
    // fresh allocation, so a graph that captured an earlier run keeps reading
    // the image (and grid) it was captured with; all are freed by destroy
    std::vector<char *> retired;
};

namespace {

// Largest device image over the update-tile shapes (a handle keeps room for
// any of them, so autotuning can re-plan in place).
size_t batch_image_cap(const std::vector<sr::BatchDesc> &h) {
    size_t cap = 256;
    for (int t = 1; t <= 3; t++) {
        sr::BatchPlan *p = sr::batch_plan_create(h.data(), (int64_t)h.size(), t);
        if (!p) return 0;
        cap = std::max(cap, (size_t)round_up((int64_t)sr::batch_plan_bytes(p, (int64_t)h.size()), 256));
        sr::batch_plan_destroy(p);
    }
    return cap;
}

// Uploads the image of `plan` for descriptors h to dst on st and waits.
hipError_t upload_image(const sr::BatchPlan *plan, const std::vector<sr::BatchDesc> &h, void *dst,
                        hipStream_t st) {
    std::vector<char> img(sr::batch_plan_bytes(plan, (int64_t)h.size()));
    sr::batch_plan_image(plan, h.data(), (int64_t)h.size(), img.data());
    hipError_t e = hipMemcpyAsync(dst, img.data(), img.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return e;
}

int batch_create_impl(int kind, void *const *T, const int64_t *ldt, const int64_t *D,
                      int64_t count, unsigned flags, int tile, sr_batch **out, void *stream);

void batch_free(sr_batch *b) {
    if (!b) return;
    if (b->plan) sr::batch_plan_destroy(b->plan);
    if (b->dev) (void)hipFree(b->dev);
    for (char *p : b->retired) (void)hipFree(p);
    delete b;
}

}  // namespace

extern "C" {

int sr_batch_create(int kind, void *const *T, const int64_t *ldt, const int64_t *D, int64_t count,
                    unsigned flags, int tile, sr_batch **out, void *stream) {
    try {
        return batch_create_impl(kind, T, ldt, D, count, flags, tile, out, stream);
    } catch (const std::bad_alloc &) {
        if (out) *out = nullptr;
        return fail(SR_ENOMEM, "sr_batch_create: out of host memory");
    }
}

}  // extern "C"

namespace {

int batch_create_impl(int kind, void *const *T, const int64_t *ldt, const int64_t *D,
                      int64_t count, unsigned flags, int tile, sr_batch **out, void *stream) {
    if (!out) return fail(SR_EINVAL, "sr_batch_create: NULL out");
    *out = nullptr;
    if (tile < SR_BATCH_TILE_AUTO || tile > SR_BATCH_TILE_64x64)
        return fail(SR_EINVAL, "sr_batch_create: unknown tile %d", tile);
    int rc = check_batch("sr_batch_create", kind, T, ldt, D, count, flags);
    if (rc != SR_OK) return rc;
    if (batch_wide(kind) && tile != SR_BATCH_TILE_AUTO && tile != SR_BATCH_TILE_64x32)
        return fail(SR_EINVAL, "sr_batch_create: 32-bit batches have one tile shape, 64 x 32");
    hipStream_t st = as_stream(stream);
    if (capturing(st))
        return fail(SR_EUNSUPPORTED, "sr_batch_create: the stream is being captured");
    std::unique_ptr<sr_batch, void (*)(sr_batch *)> b(new sr_batch, batch_free);
    b->kind = kind;
    b->s8 = batch_in_copies(kind);
    b->bits = kind == SR_BOOL;
    b->wide = batch_wide(kind);
    b->dual = is_dist(kind);
    b->reflexive = (flags & SR_REFLEXIVE) != 0;
    b->count = count;
    if (hipGetDevice(&b->device) != hipSuccess)
        return fail(SR_EDEVICE, "sr_batch_create: no current device");
    if (count > 0) {
        b->h = batch_descs(kind, T, ldt, D, count, &b->work_elems);
        b->image_cap = batch_image_cap(b->h);
        if (!b->image_cap) return fail(SR_EINVAL, "sr_batch_create: %s", kPlanFailure);
        const size_t bytes = b->image_cap + b->work_elems * 2;
        if (hipMalloc(reinterpret_cast<void **>(&b->dev), bytes) != hipSuccess) {
            b->dev = nullptr;
            (void)hipGetLastError();
            return fail(SR_ENOMEM, "sr_batch_create: could not allocate %zu bytes", bytes);
        }
        if (b->s8) place_working_copies(b->h, b->dev + b->image_cap);
        b->plan = sr::batch_plan_create(b->h.data(), count,
                                        tile ? tile : batch_tile_for(kind, b->h));
        if (!b->plan) return fail(SR_EINVAL, "sr_batch_create: %s", kPlanFailure);
        const hipError_t e = upload_image(b->plan, b->h, b->dev, st);
        if (e != hipSuccess) return device_fail(e, "sr_batch_create upload");
        b->image = b->dev;
    }
    *out = b.release();
    return ok();
}

int batch_autotune_impl(sr_batch *b, int *chosen, void *stream);

}  // namespace

extern "C" {

int sr_batch_run(sr_batch *b, void *stream) {
    if (!b) return fail(SR_EINVAL, "sr_batch_run: NULL batch");
    if (b->count == 0) return ok();
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != b->device)
        return fail(SR_EINVAL, "sr_batch_run: the batch belongs to device %d, current is %d",
                    b->device, dev);
    const hipError_t e = sr::launch_ad_closure_batched_resident(
        b->s8, b->plan, b->count, b->image, b->dual, b->reflexive, b->bits, b->wide,
        as_stream(stream));
    if (e != hipSuccess) return device_fail(e, "sr_batch_run launch");
    return ok();
}

int sr_batch_tile(const sr_batch *b) {
    return b && b->plan ? sr::batch_plan_tile(b->plan) : SR_BATCH_TILE_AUTO;
}

int sr_batch_autotune(sr_batch *b, int *chosen, void *stream) {
    try {
        return batch_autotune_impl(b, chosen, stream);
    } catch (const std::bad_alloc &) {
        return fail(SR_ENOMEM, "sr_batch_autotune: out of host memory");
    }
}

void sr_batch_destroy(sr_batch *b) { batch_free(b); }

}  // extern "C"

namespace {

int batch_autotune_impl(sr_batch *b, int *chosen, void *stream) {
    if (!b) return fail(SR_EINVAL, "sr_batch_autotune: NULL batch");
    hipStream_t st = as_stream(stream);
    if (capturing(st))
        return fail(SR_EUNSUPPORTED, "sr_batch_autotune: the stream is being captured");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != b->device)
        return fail(SR_EINVAL, "sr_batch_autotune: the batch belongs to device %d, current is %d",
                    b->device, dev);
    if (b->count == 0) {
        if (chosen) *chosen = sr_batch_tile(b);
        return ok();
    }
    // zero matrices of the batch's sizes and strides (each 256-byte aligned),
    // then room for a plan image; uint8 and Boolean batches reuse the
    // handle's working copies
    const int64_t ub = b->s8 ? 1 : unit_bytes(b->kind);
    std::vector<size_t> offs(b->h.size());
    size_t mat_bytes = 0;
    for (size_t i = 0; i < b->h.size(); i++) {
        offs[i] = mat_bytes;
        const int64_t ld = b->s8 ? b->h[i].ld8 : b->h[i].ld;
        mat_bytes += (size_t)round_up((int64_t)b->h[i].D * ld * ub, 256);
    }
    mat_bytes = std::max<size_t>(mat_bytes, 256);
    EventPair ev;
    if (!ev.ok()) return device_fail(hipErrorOutOfMemory, "sr_batch_autotune: events");
    void *z = nullptr;
    int rc = work_alloc(&z, mat_bytes + b->image_cap, st);
    if (rc != SR_OK) return rc;
    char *zm = static_cast<char *>(z), *zimg = zm + mat_bytes;
    std::vector<sr::BatchDesc> th = b->h;
    for (size_t i = 0; i < th.size(); i++) {
        if (b->s8)
            th[i].T8 = reinterpret_cast<uint8_t *>(zm + offs[i]);
        else if (b->wide)
            th[i].T32 = reinterpret_cast<uint32_t *>(zm + offs[i]);
        else
            th[i].T = reinterpret_cast<uint16_t *>(zm + offs[i]);
    }
    int pick = 0;
    float best = 0.0f;
    for (int t = b->wide ? 2 : 1; t <= (b->wide ? 2 : 3); t++) {
        std::unique_ptr<sr::BatchPlan, void (*)(sr::BatchPlan *)> p(
            sr::batch_plan_create(th.data(), b->count, t), sr::batch_plan_destroy);
        if (!p || upload_image(p.get(), th, zimg, st) != hipSuccess) continue;
        const float ms = time_candidate(
            st, ev.a, ev.b, 2, [&] { return hipMemsetAsync(zm, 0, mat_bytes, st); },
            [&] {
                return sr::launch_ad_closure_batched_resident(b->s8, p.get(), b->count, zimg,
                                                              b->dual, b->reflexive, b->bits,
                                                              b->wide, st) ==
                               hipSuccess
                           ? SR_OK
                           : SR_EDEVICE;
            });
        if (ms >= 0.0f && (!pick || ms < best)) {
            pick = t;
            best = ms;
        }
    }
    work_free(z, st);
    (void)hipStreamSynchronize(st);
    if (!pick) return fail(SR_EDEVICE, "sr_batch_autotune: no candidate ran");
    if (pick != sr::batch_plan_tile(b->plan)) {
        // the new plan goes to a fresh image; the current one stays
        // allocated (and unchanged) for graphs captured from earlier runs
        std::unique_ptr<sr::BatchPlan, void (*)(sr::BatchPlan *)> np(
            sr::batch_plan_create(b->h.data(), b->count, pick), sr::batch_plan_destroy);
        if (!np) return fail(SR_EINVAL, "sr_batch_autotune: %s", kPlanFailure);
        const size_t bytes = (size_t)round_up(
            (int64_t)sr::batch_plan_bytes(np.get(), b->count), 256);
        char *img = nullptr;
        if (hipMalloc(reinterpret_cast<void **>(&img), bytes) != hipSuccess) {
            (void)hipGetLastError();
            return fail(SR_ENOMEM, "sr_batch_autotune: could not allocate %zu bytes", bytes);
        }
        b->retired.push_back(img);
        const hipError_t e = upload_image(np.get(), b->h, img, st);
        if (e != hipSuccess) return device_fail(e, "sr_batch_autotune upload");
        sr::batch_plan_destroy(b->plan);
        b->plan = np.release();
        b->image = img;
    }
    sr::tuned_set(sr::kTuneBatch, b->kind, b->h.front().D, b->count, 0, (unsigned)pick);
    if (chosen) *chosen = pick;
    return ok();
}

}  // namespace
