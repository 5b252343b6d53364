// Boolean product on the matrix cores: C (|)= A * B as an integer product of
// {0, 1} matrices followed by a threshold (not a step of the paper: a GPU
// alternative to the word-parallel OR of Sec. II).  For every (i, j) the
// count sum_k A_ik B_kj lies in [0, K] and is positive exactly when some
// A_ik = B_kj = 1, so "count > 0" is the Boolean product entry, exactly.
//
// Two expansion kernels turn bits into bytes -- A row-major (A8[i][k]) and
// B transposed (B8T[j][k] = B_kj), both with the inner index k contiguous --
// and the product kernel feeds 16-byte slices of those rows to
// v_mfma_i32_32x32x32_i8.  Lane layout of that instruction (checked on the
// device): lane l supplies row l % 32 of the A block and column l % 32 of the
// B block, with k = 16 (l / 32) + byte over a 32-wide k slice; result register
// r of lane l is entry (8 (r / 4) + 4 (l / 32) + r % 4, l % 32) of the 32 x 32
// block.  So one ballot of "register r > 0" over the wave is two complete
// 32-column words of C: rows 8 (r / 4) + r % 4 (lanes 0..31) and that + 4
// (lanes 32..63).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sr_internal.h"

namespace sr {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

// 4 bits -> 4 bytes of 0 / 1 (bit b to byte b).
__device__ __forceinline__ uint32_t spread4(uint32_t x) {
    return ((x & 0xFu) * 0x00204081u) & 0x01010101u;
}

// A8[i][k] = bit k of row i of A, for i < rows_pad, k < kp (zero outside R x K).
// One thread per 16 bytes.
__global__ void __launch_bounds__(256)
k_expand_rows(uint8_t *A8, int64_t kp, const uint32_t *A, int64_t lda, int64_t R, int64_t K,
              int64_t rows_pad) {
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t gpr = kp / 16;
    if (g >= rows_pad * gpr) return;
    const int64_t i = g / gpr, k0 = (g % gpr) * 16;
    uint32_t bits = 0;
    if (i < R && k0 < K) {
        bits = (A[i * lda + (k0 >> 5)] >> (k0 & 31)) & 0xFFFFu;
        if (K - k0 < 16) bits &= (1u << (K - k0)) - 1u;
    }
    uint4 o;
    o.x = spread4(bits);
    o.y = spread4(bits >> 4);
    o.z = spread4(bits >> 8);
    o.w = spread4(bits >> 12);
    *reinterpret_cast<uint4 *>(A8 + i * kp + k0) = o;
}

// B8T[j][k] = bit j of row k of B, for j < cols_pad, k < kp (zero outside
// K x N).  One thread per 16 bytes (16 rows of B, one column).
__global__ void __launch_bounds__(256)
k_expand_cols(uint8_t *B8T, int64_t kp, const uint32_t *B, int64_t ldb, int64_t K, int64_t N,
              int64_t cols_pad) {
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t gpr = kp / 16;
    if (g >= cols_pad * gpr) return;
    // consecutive threads take consecutive columns of one 16-row group, so a
    // wave reads two words per row of B
    const int64_t j = g % cols_pad, k0 = (g / cols_pad) * 16;
    uint32_t v[4] = {0u, 0u, 0u, 0u};
    if (j < N) {
        const uint32_t *col = B + (j >> 5);
        const int sh = (int)(j & 31);
#pragma unroll
        for (int b = 0; b < 16; b++) {
            const int64_t k = k0 + b;
            const uint32_t bit = k < K ? (col[k * ldb] >> sh) & 1u : 0u;
            v[b >> 2] |= bit << (8 * (b & 3));
        }
    }
    *reinterpret_cast<uint4 *>(B8T + j * kp + k0) = uint4{v[0], v[1], v[2], v[3]};
}

// Lane `at` of the result takes the wave-uniform value v; other lanes keep w.
__device__ __forceinline__ uint32_t put_lane(uint32_t w, uint32_t v, int at, int lane) {
    return lane == at ? v : w;
}

// C (|)= A * B over a 128 x 128 tile per workgroup: wave w takes rows
// 64 (w / 2) .. +64 and columns 64 (w % 2) .. +64 of the tile as 2 x 2 blocks of
// 32 x 32.  kp: inner bytes per row of A8 / B8T (a multiple of 64).
__global__ void __launch_bounds__(256)
k_bool_mul_mfma(uint32_t *C, int64_t ldc, const uint8_t *A8, const uint8_t *B8T, int64_t kp,
                int64_t R, int64_t N, int accumulate) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t row0 = (int64_t)blockIdx.y * 128 + 64 * (wave >> 1);
    const int64_t col0 = (int64_t)blockIdx.x * 128 + 64 * (wave & 1);
    if (row0 >= R || col0 >= N) return;
    if (kp == 0) return;  // no inner index: the host never launches this case
    const int half = 16 * (lane >> 5);
    const uint8_t *a0 = A8 + (row0 + (lane & 31)) * kp + half;
    const uint8_t *a1 = a0 + 32 * kp;
    const uint8_t *b0 = B8T + (col0 + (lane & 31)) * kp + half;
    const uint8_t *b1 = b0 + 32 * kp;
    v16i acc00 = {}, acc01 = {}, acc10 = {}, acc11 = {};
    // Two slices of 32 per iteration; each slice's operands are requested one
    // slice ahead of their use (vector loads return in order, so the waits
    // are partial).  Requests past the end re-read the last slice.
    auto ld = [&](const uint8_t *p, int64_t k) {
        return *reinterpret_cast<const v4i *>(p + (k < kp ? k : kp - 32));
    };
    v4i xa0 = ld(a0, 0), xa1 = ld(a1, 0), xb0 = ld(b0, 0), xb1 = ld(b1, 0);
    __builtin_amdgcn_sched_barrier(0);
    v4i ya0 = ld(a0, 32), ya1 = ld(a1, 32), yb0 = ld(b0, 32), yb1 = ld(b1, 32);
    __builtin_amdgcn_sched_barrier(0);
    // (the scheduling barriers keep the compiler from sinking each request
    // down to its use)
    for (int64_t k = 0; k < kp; k += 64) {
        acc00 = __builtin_amdgcn_mfma_i32_32x32x32_i8(xa0, xb0, acc00, 0, 0, 0);
        acc01 = __builtin_amdgcn_mfma_i32_32x32x32_i8(xa0, xb1, acc01, 0, 0, 0);
        acc10 = __builtin_amdgcn_mfma_i32_32x32x32_i8(xa1, xb0, acc10, 0, 0, 0);
        acc11 = __builtin_amdgcn_mfma_i32_32x32x32_i8(xa1, xb1, acc11, 0, 0, 0);
        __builtin_amdgcn_sched_barrier(0);
        xa0 = ld(a0, k + 64), xa1 = ld(a1, k + 64), xb0 = ld(b0, k + 64), xb1 = ld(b1, k + 64);
        __builtin_amdgcn_sched_barrier(0);
        acc00 = __builtin_amdgcn_mfma_i32_32x32x32_i8(ya0, yb0, acc00, 0, 0, 0);
        acc01 = __builtin_amdgcn_mfma_i32_32x32x32_i8(ya0, yb1, acc01, 0, 0, 0);
        acc10 = __builtin_amdgcn_mfma_i32_32x32x32_i8(ya1, yb0, acc10, 0, 0, 0);
        acc11 = __builtin_amdgcn_mfma_i32_32x32x32_i8(ya1, yb1, acc11, 0, 0, 0);
        __builtin_amdgcn_sched_barrier(0);
        ya0 = ld(a0, k + 96), ya1 = ld(a1, k + 96), yb0 = ld(b0, k + 96), yb1 = ld(b1, k + 96);
        __builtin_amdgcn_sched_barrier(0);
    }
    // threshold and repack: word c of lane L = bits of row row0 + L, columns
    // col0 + 32 c .. +32
    uint32_t w0 = 0u, w1 = 0u;
#pragma unroll
    for (int r = 0; r < 16; r++) {
        const int i0 = 8 * (r / 4) + (r % 4);
        const uint64_t m00 = __builtin_amdgcn_ballot_w64(acc00[r] > 0);
        const uint64_t m01 = __builtin_amdgcn_ballot_w64(acc01[r] > 0);
        const uint64_t m10 = __builtin_amdgcn_ballot_w64(acc10[r] > 0);
        const uint64_t m11 = __builtin_amdgcn_ballot_w64(acc11[r] > 0);
        w0 = put_lane(w0, (uint32_t)m00, i0, lane);
        w0 = put_lane(w0, (uint32_t)(m00 >> 32), i0 + 4, lane);
        w1 = put_lane(w1, (uint32_t)m01, i0, lane);
        w1 = put_lane(w1, (uint32_t)(m01 >> 32), i0 + 4, lane);
        w0 = put_lane(w0, (uint32_t)m10, 32 + i0, lane);
        w0 = put_lane(w0, (uint32_t)(m10 >> 32), 32 + i0 + 4, lane);
        w1 = put_lane(w1, (uint32_t)m11, 32 + i0, lane);
        w1 = put_lane(w1, (uint32_t)(m11 >> 32), 32 + i0 + 4, lane);
    }
    const int64_t row = row0 + lane;
    if (row >= R) return;
    uint32_t *crow = C + row * ldc + (col0 >> 5);
    if (accumulate) {
        crow[0] |= w0;
        if (col0 + 32 < N) crow[1] |= w1;
    } else {
        crow[0] = w0;
        if (col0 + 32 < N) crow[1] = w1;
    }
}

}  // namespace

size_t bool_mfma_work_bytes(int64_t R, int64_t K, int64_t N) {
    const int64_t kp = (K + 63) / 64 * 64;
    const int64_t rp = (R + 127) / 128 * 128, np = (N + 127) / 128 * 128;
    return (size_t)(rp + np) * (size_t)kp;
}

hipError_t launch_bool_mul_mfma(uint64_t *C, int64_t ldc, const uint64_t *A, int64_t lda,
                                const uint64_t *B, int64_t ldb, int64_t R, int64_t K, int64_t N,
                                bool accumulate, void *work, hipStream_t st) {
    // K = 0: the product is the zero matrix; the operand loads of the
    // product kernel need at least one 64-byte slice, so this case goes to
    // the bit-sliced kernels (which write the zeros, or leave C as it is)
    if (K == 0)
        return launch_bool_mul(C, ldc, A, lda, B, ldb, R, K, N, accumulate, kBoolPathBitwise, st);
    const int64_t kp = (K + 63) / 64 * 64;
    const int64_t rp = (R + 127) / 128 * 128, np = (N + 127) / 128 * 128;
    uint8_t *A8 = static_cast<uint8_t *>(work);
    uint8_t *B8T = A8 + rp * kp;
    const uint32_t *a = reinterpret_cast<const uint32_t *>(A);
    const uint32_t *b = reinterpret_cast<const uint32_t *>(B);
    if (kp > 0) {
        const int64_t ta = rp * (kp / 16), tb = np * (kp / 16);
        hipLaunchKernelGGL(k_expand_rows, dim3((unsigned)((ta + 255) / 256)), dim3(256), 0, st, A8,
                           kp, a, 2 * lda, R, K, rp);
        hipLaunchKernelGGL(k_expand_cols, dim3((unsigned)((tb + 255) / 256)), dim3(256), 0, st,
                           B8T, kp, b, 2 * ldb, K, N, np);
    }
    hipLaunchKernelGGL(k_bool_mul_mfma, dim3((unsigned)(np / 128), (unsigned)(rp / 128)), dim3(256),
                       0, st, reinterpret_cast<uint32_t *>(C), 2 * ldc, A8, B8T, kp, R, N,
                       accumulate ? 1 : 0);
    return hipGetLastError();
}

}  // namespace sr
