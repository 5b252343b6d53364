// Entrywise operations of the table in Sec. V -- and = min, or = max (the
// matrix (+) of Sec. II), xor = |a - b|, not = S - a -- on anti-distance or
// distance entries (uint8 / uint16 / uint32, where S - a is the bitwise
// complement) and
// on Boolean words (AND, OR, XOR, NOT with the padding bits kept zero).  One
// thread per 16-byte group of a row; HBM-bound.  Operands too large to stay
// in the caches are read and written with the nontemporal hint (the
// streaming form: 76.9 -> 62.0 us at 8192 x 8192 uint16, 5.2 -> 6.5 TB/s); small
// ones keep the default policy, since the next kernel usually reads the
// result.  Also the diagonal write of the reflexive closure I (+) T (eq. rtc).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "sr_internal.h"

namespace sr {
namespace {

typedef uint8_t u8x4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// 16-byte load / store, with the nontemporal hint when NT.
template <bool NT>
__device__ __forceinline__ u32x4 load16(const uint8_t *p) {
    const u32x4 *q = reinterpret_cast<const u32x4 *>(p);
    if (NT) return __builtin_nontemporal_load(q);
    return *q;
}
template <bool NT>
__device__ __forceinline__ void store16(uint8_t *p, u32x4 v) {
    u32x4 *q = reinterpret_cast<u32x4 *>(p);
    if (NT)
        __builtin_nontemporal_store(v, q);
    else
        *q = v;
}

template <typename V>
__device__ __forceinline__ uint32_t lanes_op(int op, uint32_t a, uint32_t b) {
    const V x = __builtin_bit_cast(V, a), y = __builtin_bit_cast(V, b);
    V r;
    if (op == EW_AND)
        r = __builtin_elementwise_min(x, y);
    else if (op == EW_OR)
        r = __builtin_elementwise_max(x, y);
    else  // EW_XOR: |a - b|
        r = __builtin_elementwise_max(x, y) - __builtin_elementwise_min(x, y);
    return __builtin_bit_cast(uint32_t, r);
}

// One 32-bit word of a row: OP on entries of ES bytes (1, 2, 4) or on bits (8).
template <int ES, int OP>
__device__ __forceinline__ uint32_t op_word(uint32_t a, uint32_t b) {
    if (OP == EW_NOT) return ~a;
    if (ES == 1) return lanes_op<u8x4>(OP, a, b);
    if (ES == 2) return lanes_op<u16x2>(OP, a, b);
    if (ES == 4) {
        const uint32_t lo = min(a, b), hi = max(a, b);
        return OP == EW_AND ? lo : (OP == EW_OR ? hi : hi - lo);
    }
    return OP == EW_AND ? (a & b) : (OP == EW_OR ? (a | b) : (a ^ b));
}

// Row strides in bytes (multiples of 16); nbytes = valid bytes per row;
// nbits (Boolean NOT only): valid bits per row, the rest of the row's words
// are written as zero.
template <int ES, int OP, bool NT>
__global__ void __launch_bounds__(256)
k_ewise(uint8_t *C, int64_t ldc, const uint8_t *A, int64_t lda, const uint8_t *B, int64_t ldb,
        int64_t R, int64_t nbytes, int64_t nbits) {
    const int64_t gpr = (nbytes + 15) >> 4;
    const int64_t total = R * gpr;
    for (int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x; g < total;
         g += (int64_t)gridDim.x * 256) {
        const int64_t row = g / gpr, b0 = (g % gpr) * 16;
        const u32x4 a = load16<NT>(A + row * lda + b0);
        u32x4 b = a;
        if (OP != EW_NOT) b = load16<NT>(B + row * ldb + b0);
        uint32_t cw[4] = {op_word<ES, OP>(a.x, b.x), op_word<ES, OP>(a.y, b.y),
                          op_word<ES, OP>(a.z, b.z), op_word<ES, OP>(a.w, b.w)};
        if (ES == 8 && OP == EW_NOT) {
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const int64_t first = 8 * (b0 + 4 * q);  // first bit of this word
                const int64_t valid = nbits - first;
                if (valid <= 0)
                    cw[q] = 0u;
                else if (valid < 32)
                    cw[q] &= (1u << valid) - 1u;
            }
        }
        uint8_t *dst = C + row * ldc + b0;
        if (b0 + 16 <= nbytes) {
            store16<NT>(dst, u32x4{cw[0], cw[1], cw[2], cw[3]});
        } else {
            for (int i = 0; i < 16 && b0 + i < nbytes; i++)
                dst[i] = (uint8_t)(cw[i >> 2] >> (8 * (i & 3)));
        }
    }
}

template <int ES, bool NT>
hipError_t ewise_es(int op, uint8_t *c, int64_t ldcb, const uint8_t *a, int64_t ldab,
                    const uint8_t *b, int64_t ldbb, int64_t R, int64_t nbytes, int64_t nbits,
                    unsigned blocks, hipStream_t st) {
    switch (op) {
        case EW_AND:
            hipLaunchKernelGGL((k_ewise<ES, EW_AND, NT>), dim3(blocks), dim3(256), 0, st, c, ldcb,
                               a, ldab, b, ldbb, R, nbytes, nbits);
            break;
        case EW_OR:
            hipLaunchKernelGGL((k_ewise<ES, EW_OR, NT>), dim3(blocks), dim3(256), 0, st, c, ldcb,
                               a, ldab, b, ldbb, R, nbytes, nbits);
            break;
        case EW_XOR:
            hipLaunchKernelGGL((k_ewise<ES, EW_XOR, NT>), dim3(blocks), dim3(256), 0, st, c, ldcb,
                               a, ldab, b, ldbb, R, nbytes, nbits);
            break;
        default:
            hipLaunchKernelGGL((k_ewise<ES, EW_NOT, NT>), dim3(blocks), dim3(256), 0, st, c, ldcb,
                               a, ldab, b, ldbb, R, nbytes, nbits);
            break;
    }
    return hipGetLastError();
}

template <int ES>
hipError_t ewise_nt(bool nt, int op, uint8_t *c, int64_t ldcb, const uint8_t *a, int64_t ldab,
                    const uint8_t *b, int64_t ldbb, int64_t R, int64_t nbytes, int64_t nbits,
                    unsigned blocks, hipStream_t st) {
    return nt ? ewise_es<ES, true>(op, c, ldcb, a, ldab, b, ldbb, R, nbytes, nbits, blocks, st)
              : ewise_es<ES, false>(op, c, ldcb, a, ldab, b, ldbb, R, nbytes, nbits, blocks, st);
}

// Diagonal of a D x D matrix: entries set to `value` (ES = 1, 2, 4), or bit i of
// row i set (ES = 8, Boolean words).  One thread per row.
template <int ES>
__global__ void __launch_bounds__(256) k_diag(uint8_t *T, int64_t ldb, int64_t D, uint32_t value) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= D) return;
    uint8_t *row = T + i * ldb;
    if (ES == 1)
        row[i] = (uint8_t)value;
    else if (ES == 2)
        reinterpret_cast<uint16_t *>(row)[i] = (uint16_t)value;
    else if (ES == 4)
        reinterpret_cast<uint32_t *>(row)[i] = value;
    else
        reinterpret_cast<uint32_t *>(row)[i >> 5] |= 1u << (i & 31);
}

// p[0 .. n) := value, grid-stride over 32-bit words.
__global__ void __launch_bounds__(256) k_fill32(uint32_t *p, int64_t n, uint32_t value) {
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) p[i] = value;
}

}  // namespace

hipError_t launch_ewise(int elem_bytes, int op, void *C, int64_t ldc, const void *A, int64_t lda,
                        const void *B, int64_t ldb, int64_t R, int64_t N, int64_t nbits,
                        hipStream_t stream) {
    const int64_t nbytes = N * elem_bytes;
    const int64_t groups = R * ((nbytes + 15) / 16);
    if (groups == 0) return hipSuccess;
    // one group per thread up to 65536 workgroups (8192 x 8192 uint16 takes
    // 32768), grid-stride beyond
    const unsigned blocks = (unsigned)std::min<int64_t>((groups + 255) / 256, 65536);
    // streaming hint once one operand exceeds 16 MiB (the 32 MiB of L2 could
    // not hold the three)
    const bool nt = groups >= (int64_t(16) << 20) / 16;
    uint8_t *c = static_cast<uint8_t *>(C);
    const uint8_t *a = static_cast<const uint8_t *>(A);
    const uint8_t *b = static_cast<const uint8_t *>(B);
    const int64_t e = elem_bytes;
    switch (elem_bytes) {
        case 1: return ewise_nt<1>(nt, op, c, ldc * e, a, lda * e, b, ldb * e, R, nbytes, nbits, blocks, stream);
        case 2: return ewise_nt<2>(nt, op, c, ldc * e, a, lda * e, b, ldb * e, R, nbytes, nbits, blocks, stream);
        case 4: return ewise_nt<4>(nt, op, c, ldc * e, a, lda * e, b, ldb * e, R, nbytes, nbits, blocks, stream);
        default: return ewise_nt<8>(nt, op, c, ldc * e, a, lda * e, b, ldb * e, R, nbytes, nbits, blocks, stream);
    }
}

hipError_t launch_add(int elem_bytes, void *C, int64_t ldc, const void *A, int64_t lda,
                      const void *B, int64_t ldb, int64_t R, int64_t N, hipStream_t stream) {
    return launch_ewise(elem_bytes, EW_OR, C, ldc, A, lda, B, ldb, R, N, 0, stream);
}

hipError_t launch_diag(int elem_bytes, void *T, int64_t ld, int64_t D, uint32_t value,
                       hipStream_t stream) {
    if (D <= 0) return hipSuccess;
    const dim3 grid((unsigned)((D + 255) / 256));
    uint8_t *t = static_cast<uint8_t *>(T);
    const int64_t ldb = ld * elem_bytes;
    switch (elem_bytes) {
        case 1: hipLaunchKernelGGL(k_diag<1>, grid, dim3(256), 0, stream, t, ldb, D, value); break;
        case 2: hipLaunchKernelGGL(k_diag<2>, grid, dim3(256), 0, stream, t, ldb, D, value); break;
        case 4: hipLaunchKernelGGL(k_diag<4>, grid, dim3(256), 0, stream, t, ldb, D, value); break;
        default: hipLaunchKernelGGL(k_diag<8>, grid, dim3(256), 0, stream, t, ldb, D, value); break;
    }
    return hipGetLastError();
}

hipError_t launch_fill32(uint32_t *p, int64_t n, uint32_t value, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 2048);
    hipLaunchKernelGGL(k_fill32, dim3((unsigned)blocks), dim3(256), 0, stream, p, n, value);
    return hipGetLastError();
}

}  // namespace sr
