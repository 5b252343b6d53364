// Entrywise (+) of two matrices (Sec. II matrix addition; the `|` operator of
// the entrywise table in Sec. V): max for anti-distance entries, OR for
// Boolean words.  One thread per 16-byte group of a row; HBM-bound.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sr_internal.h"

namespace sr {
namespace {

typedef uint8_t u8x4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16x2 __attribute__((ext_vector_type(2)));

template <int ES>
__device__ __forceinline__ uint32_t op_word(uint32_t a, uint32_t b) {
    if (ES == 1)
        return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(u8x4, a),
                                                                      __builtin_bit_cast(u8x4, b)));
    if (ES == 2)
        return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(u16x2, a),
                                                                      __builtin_bit_cast(u16x2, b)));
    return a | b;
}

// Row strides in bytes (multiples of 16); nbytes = valid bytes per row.
template <int ES>
__global__ void __launch_bounds__(256)
k_add(uint8_t *C, int64_t ldc, const uint8_t *A, int64_t lda, const uint8_t *B, int64_t ldb,
      int64_t R, int64_t nbytes) {
    const int64_t gpr = (nbytes + 15) >> 4;
    const int64_t total = R * gpr;
    for (int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x; g < total;
         g += (int64_t)gridDim.x * 256) {
        const int64_t row = g / gpr, b0 = (g % gpr) * 16;
        const uint4 a = *reinterpret_cast<const uint4 *>(A + row * lda + b0);
        const uint4 b = *reinterpret_cast<const uint4 *>(B + row * ldb + b0);
        uint4 c;
        c.x = op_word<ES>(a.x, b.x);
        c.y = op_word<ES>(a.y, b.y);
        c.z = op_word<ES>(a.z, b.z);
        c.w = op_word<ES>(a.w, b.w);
        uint8_t *dst = C + row * ldc + b0;
        if (b0 + 16 <= nbytes) {
            *reinterpret_cast<uint4 *>(dst) = c;
        } else {
            const uint32_t cw[4] = {c.x, c.y, c.z, c.w};
            for (int i = 0; i < 16 && b0 + i < nbytes; i++)
                dst[i] = (uint8_t)(cw[i >> 2] >> (8 * (i & 3)));
        }
    }
}

}  // namespace

hipError_t launch_add(int elem_bytes, void *C, int64_t ldc, const void *A, int64_t lda,
                      const void *B, int64_t ldb, int64_t R, int64_t N, hipStream_t stream) {
    const int64_t nbytes = N * elem_bytes;
    const int64_t groups = R * ((nbytes + 15) / 16);
    if (groups == 0) return hipSuccess;
    const int64_t blocks = groups < 256 * 2048 ? (groups + 255) / 256 : 2048;
    uint8_t *c = static_cast<uint8_t *>(C);
    const uint8_t *a = static_cast<const uint8_t *>(A);
    const uint8_t *b = static_cast<const uint8_t *>(B);
    const int64_t e = elem_bytes;
    switch (elem_bytes) {
        case 1:
            hipLaunchKernelGGL(k_add<1>, dim3((unsigned)blocks), dim3(256), 0, stream, c, ldc * e, a,
                               lda * e, b, ldb * e, R, nbytes);
            break;
        case 2:
            hipLaunchKernelGGL(k_add<2>, dim3((unsigned)blocks), dim3(256), 0, stream, c, ldc * e, a,
                               lda * e, b, ldb * e, R, nbytes);
            break;
        default:
            hipLaunchKernelGGL(k_add<8>, dim3((unsigned)blocks), dim3(256), 0, stream, c, ldc * e, a,
                               lda * e, b, ldb * e, R, nbytes);
            break;
    }
    return hipGetLastError();
}

}  // namespace sr
