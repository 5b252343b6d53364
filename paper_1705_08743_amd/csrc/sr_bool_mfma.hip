// Boolean product on the matrix cores: C (|)= A * B as a count of common
// set bits followed by a threshold (not a step of the paper: a GPU
// alternative to the word-parallel OR of Sec. II).  For every (i, j) the
// count sum_k A_ik B_kj lies in [0, K] and is positive exactly when some
// A_ik = B_kj = 1, so "count > 0" is the Boolean product entry, exactly.
//
// Operands come straight from the packed bits, with no expanded copy in
// memory.  A wave multiplies 32 x 32 blocks; lane l supplies row l % 32 of
// its A block and column l % 32 of its B block, and the two lane halves
// supply the two halves of the inner slice.  Since the sum over k does not
// depend on the order of the inner index, the inner index may be laid out in
// the operand registers in any order, as long as A and B use the same one.
// Each lane therefore takes one 32-bit word of its packed row (A) or of its
// packed column (B, from a bit-transposed copy: word w of row j of BT holds
// B_kj for k = 32w .. 32w + 31) and spreads its bits over the operand with a
// few masks:
//
//   F4 (v_mfma_scale_f32_32x32x64_f8f6f4 on 4-bit e2m1 values, unit
//   scales): the 32 nibbles of the operand are x & 0x11111111,
//   x & 0x22222222, x & 0x44444444 and (x >> 1) & 0x44444444, i.e. one bit per
//   nibble at a position that makes it 0.5, 1 or 2 (never the sign bit), so a
//   product of two set bits is 0.25 .. 4 and the fp32 sum of at most K such
//   terms (all multiples of 0.25, below 2^18 for K <= 65536) is exact and
//   positive exactly when the count is.
//   I8 (v_mfma_i32_32x32x32_i8): two operands per word, byte e of dword d
//   = bit 8e + d of x (d = 0..3), then bit 8e + 4 + d: values 0 / 1, int32
//   counts.
//
// The result layout (checked on the device for both forms): register r of
// lane l is entry (8 (r / 4) + 4 (l / 32) + r % 4, l % 32) of the block.  The
// wave computes the transposed blocks, B^T A^T (the packed columns of B as the
// first operand), so lane l holds 16 entries of ROW l % 32 of C, at columns
// 8 (r / 4) + 4 (l / 32) + r % 4: each lane packs its thresholds into the
// bits of its row's word, and one swap of the two lane halves
// (v_permlane32_swap) completes the word in every lane.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <stdlib.h>
#include <string.h>

#include <algorithm>

#include "sr_internal.h"

namespace sr {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef float v16f __attribute__((ext_vector_type(16)));

constexpr int kF4 = 0, kI8 = 1;

// E8M0 scale 2^0 in each of the four bytes
constexpr int kUnitScale = 0x7F7F7F7F;

template <int F>
struct Acc;
template <>
struct Acc<kF4> {
    typedef v16f type;
};
template <>
struct Acc<kI8> {
    typedef v16i type;
};

// acc += (bits of a) x (bits of b) over the 32 inner indices of one word per
// lane (see the file comment for the layout).
template <int F>
__device__ __forceinline__ void mac_word(typename Acc<F>::type &acc, uint32_t a, uint32_t b) {
    if constexpr (F == kF4) {
        const v8i x = {(int)(a & 0x11111111u), (int)(a & 0x22222222u), (int)(a & 0x44444444u),
                       (int)((a >> 1) & 0x44444444u), 0, 0, 0, 0};
        const v8i y = {(int)(b & 0x11111111u), (int)(b & 0x22222222u), (int)(b & 0x44444444u),
                       (int)((b >> 1) & 0x44444444u), 0, 0, 0, 0};
        acc = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(x, y, acc, 4, 4, 0, kUnitScale, 0,
                                                              kUnitScale);
    } else {
        const v4i x0 = {(int)(a & 0x01010101u), (int)((a >> 1) & 0x01010101u),
                        (int)((a >> 2) & 0x01010101u), (int)((a >> 3) & 0x01010101u)};
        const v4i y0 = {(int)(b & 0x01010101u), (int)((b >> 1) & 0x01010101u),
                        (int)((b >> 2) & 0x01010101u), (int)((b >> 3) & 0x01010101u)};
        acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(x0, y0, acc, 0, 0, 0);
        const v4i x1 = {(int)((a >> 4) & 0x01010101u), (int)((a >> 5) & 0x01010101u),
                        (int)((a >> 6) & 0x01010101u), (int)((a >> 7) & 0x01010101u)};
        const v4i y1 = {(int)((b >> 4) & 0x01010101u), (int)((b >> 5) & 0x01010101u),
                        (int)((b >> 6) & 0x01010101u), (int)((b >> 7) & 0x01010101u)};
        acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(x1, y1, acc, 0, 0, 0);
    }
}

__device__ __forceinline__ uint32_t as_u32(float x) { return __float_as_uint(x); }
__device__ __forceinline__ uint32_t as_u32(int x) { return (uint32_t)x; }

// Word of row l % 32 of a block from its transposed accumulator (see the file
// comment): bit c is 1 exactly when the count at column c is positive.  The
// counts are non-negative (int32, or fp32 sums of non-negative products that
// never form -0), so "positive" is min(bits, 1) of the 32-bit pattern.
template <typename V>
__device__ __forceinline__ uint32_t row_word(const V &acc, int h) {
    uint32_t bits = 0u;
#pragma unroll
    for (int r = 0; r < 16; r++)
        bits |= min(as_u32(acc[r]), 1u) << (8 * (r / 4) + (r % 4));
    bits <<= 4 * h;
    const auto sw = __builtin_amdgcn_permlane32_swap(bits, bits, false, false);
    return sw[0] | sw[1];
}

// v with lane L replaced by the wave-uniform x (v_writelane; the lane index
// is a constant).  x comes straight from a vector compare (a ballot), whose
// scalar result v_writelane may not read for a few cycles; the compiler does
// not insert those wait states for an asm statement, so it carries them
// (measured: without them each write read the previous compare's mask).
template <int L, bool WAIT>
__device__ __forceinline__ uint32_t write_lane(uint32_t v, uint32_t x) {
    if constexpr (WAIT)
        asm("s_nop 4\n\tv_writelane_b32 %0, %1, %2" : "+v"(v) : "s"(x), "i"(L));
    else
        asm("v_writelane_b32 %0, %1, %2" : "+v"(v) : "s"(x), "i"(L));
    return v;
}

// The two halves of a 64-lane ballot m into lanes LO and HI of v (the high
// half is read after the low half's write, past the wait).
template <int LO, int HI>
__device__ __forceinline__ uint32_t put_mask(uint32_t v, uint64_t m) {
    v = write_lane<LO, true>(v, (uint32_t)m);
    return write_lane<HI, false>(v, (uint32_t)(m >> 32));
}

// Four consecutive words of a packed row, from word w of p; words at or past
// nw read as zero (the last, partial group of a row).
__device__ __forceinline__ uint4 load4(const uint32_t *p, int64_t w, int64_t nw) {
    if (w + 4 <= nw) return *reinterpret_cast<const uint4 *>(p + w);
    uint4 v;
    v.x = w < nw ? p[w] : 0u;
    v.y = w + 1 < nw ? p[w + 1] : 0u;
    v.z = w + 2 < nw ? p[w + 2] : 0u;
    v.w = w + 3 < nw ? p[w + 3] : 0u;
    return v;
}

// One wave: C (|)= A * B over a tile of 64 rows x 32 BJ columns (2 x BJ
// blocks of 32 x 32).  A: the tile's first row, word 0 of its inner range
// (row stride lda, nwa words readable per row); BT: the tile's first
// column's row of the transposed B (stride ldbt, ngroups * 8 words readable
// and zero past the inner extent); C: row 0, word 0 of the tile (nrows <= 64
// rows, nwc <= BJ words stored).  Rows of A past nrows re-read the last row.
template <int F, int BJ>
__device__ __forceinline__ void mfma_tile(uint32_t *C, int64_t ldc, const uint32_t *A,
                                          int64_t lda, int64_t nwa, const uint32_t *BT,
                                          int64_t ldbt, int ngroups, int nrows, int nwc,
                                          bool accumulate) {
    const int lane = threadIdx.x & 63;
    const int h = lane >> 5, r32 = lane & 31;
    typedef typename Acc<F>::type acc_t;
    acc_t acc[2][BJ];
#pragma unroll
    for (int bi = 0; bi < 2; bi++)
#pragma unroll
        for (int bj = 0; bj < BJ; bj++) acc[bi][bj] = acc_t{};
    const uint32_t *ap[2];
#pragma unroll
    for (int bi = 0; bi < 2; bi++) ap[bi] = A + (int64_t)min(32 * bi + r32, nrows - 1) * lda;
    const uint32_t *bp[BJ];
#pragma unroll
    for (int bj = 0; bj < BJ; bj++) bp[bj] = BT + (int64_t)(32 * bj + r32) * ldbt + 4 * h;
    // group g: the lane's words 8g + 4h .. + 3 of its row / column; the next
    // group's words are requested before this group's products
    uint4 xa[2], xb[BJ];
#pragma unroll
    for (int bi = 0; bi < 2; bi++) xa[bi] = load4(ap[bi], 4 * h, nwa);
#pragma unroll
    for (int bj = 0; bj < BJ; bj++) xb[bj] = *reinterpret_cast<const uint4 *>(bp[bj]);
    for (int g = 0; g < ngroups; g++) {
        uint4 ya[2], yb[BJ];
        const int gn = g + 1 < ngroups ? g + 1 : g;
#pragma unroll
        for (int bi = 0; bi < 2; bi++) ya[bi] = load4(ap[bi], 8 * gn + 4 * h, nwa);
#pragma unroll
        for (int bj = 0; bj < BJ; bj++) yb[bj] = *reinterpret_cast<const uint4 *>(bp[bj] + 8 * gn);
#pragma unroll
        for (int u = 0; u < 4; u++) {
#pragma unroll
            for (int bi = 0; bi < 2; bi++) {
                const uint32_t a = u == 0 ? xa[bi].x : u == 1 ? xa[bi].y : u == 2 ? xa[bi].z : xa[bi].w;
#pragma unroll
                for (int bj = 0; bj < BJ; bj++) {
                    const uint32_t b =
                        u == 0 ? xb[bj].x : u == 1 ? xb[bj].y : u == 2 ? xb[bj].z : xb[bj].w;
                    mac_word<F>(acc[bi][bj], b, a);  // B^T A^T: rows of C in the lanes
                }
            }
        }
#pragma unroll
        for (int bi = 0; bi < 2; bi++) xa[bi] = ya[bi];
#pragma unroll
        for (int bj = 0; bj < BJ; bj++) xb[bj] = yb[bj];
    }
    // threshold: word bj of lane L = bits of tile row L (block row L / 32),
    // columns 32 bj .. +32
    uint32_t w[BJ];
#pragma unroll
    for (int bj = 0; bj < BJ; bj++) {
        const uint32_t w0 = row_word(acc[0][bj], h), w1 = row_word(acc[1][bj], h);
        w[bj] = h ? w1 : w0;
    }
    if (lane >= nrows) return;
    uint32_t *crow = C + (int64_t)lane * ldc;
    if (nwc == BJ && BJ % 2 == 0) {
#pragma unroll
        for (int bj = 0; bj < BJ; bj += 2) {
            uint2 v = uint2{w[bj], w[bj + 1]};
            if (accumulate) {
                const uint2 o = reinterpret_cast<const uint2 *>(crow)[bj / 2];
                v.x |= o.x;
                v.y |= o.y;
            }
            reinterpret_cast<uint2 *>(crow)[bj / 2] = v;
        }
    } else {
#pragma unroll
        for (int bj = 0; bj < BJ; bj++)
            if (bj < nwc) crow[bj] = accumulate ? (crow[bj] | w[bj]) : w[bj];
    }
}

// C (|)= A * B: workgroup = 4 waves, wave w takes rows 64 (4 y + w) .. +64 of
// columns 32 BJ x .. +32 BJ.  nwa: readable words per row of A; ngroups:
// 8-word groups of the inner index (BT's padded width / 8).
template <int F, int BJ>
__global__ void __launch_bounds__(256)
k_bool_mul_mfma(uint32_t *C, int64_t ldc, const uint32_t *A, int64_t lda, int64_t nwa,
                const uint32_t *BT, int64_t ldbt, int ngroups, int64_t R, int64_t nwords,
                int accumulate) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t row0 = ((int64_t)blockIdx.y * 4 + wave) * 64;
    const int64_t w0 = (int64_t)blockIdx.x * BJ;
    if (row0 >= R) return;
    mfma_tile<F, BJ>(C + row0 * ldc + w0, ldc, A + row0 * lda, lda, nwa, BT + 32 * w0 * ldbt,
                     ldbt, ngroups, (int)min<int64_t>(64, R - row0),
                     (int)min<int64_t>(BJ, nwords - w0), accumulate != 0);
}

// The ballot of bit B of every lane's x, for B .. 31: the low half (lanes
// 0..31) goes to lane B, the high half to lane 32 + B.
template <int B>
__device__ __forceinline__ uint32_t transpose_bits(uint32_t o, uint32_t x) {
    if constexpr (B < 32) {
        o = put_mask<B, 32 + B>(o, __builtin_amdgcn_ballot_w64((x >> B) & 1u));
        return transpose_bits<B + 1>(o, x);
    } else {
        return o;
    }
}

// Bit transpose: BT[j][w] bit t = B[32 w + t][j] for j < n_rows_bt, w <
// KW * gridDim.y words; zero where 32 w + t >= K or column j of B is past its
// nwb words.  A wave takes 64 columns (two words of B: lane half h reads word
// 2 c + h of 32 rows) and KW consecutive words of BT: each ballot over the 32
// rows of one bit position is one word for one column, sent to the lane of
// its column with v_writelane.  KW = 1 spreads a small transpose over more
// waves; KW = 4 stores 16 bytes per lane for a large one.
template <int KW>
__global__ void __launch_bounds__(256)
k_bit_transpose(uint32_t *BT, int64_t ldbt, const uint32_t *B, int64_t ldb, int64_t K,
                int64_t nwb, int64_t n_rows_bt) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t c = (int64_t)blockIdx.x * 4 + wave;  // pair of B words = 64 BT rows
    if (64 * c >= n_rows_bt) return;
    const int h = lane >> 5, t = lane & 31;
    const int64_t jw = 2 * c + h;
    const int64_t wb0 = (int64_t)blockIdx.y * KW;
    uint32_t out[KW];
#pragma unroll
    for (int kw = 0; kw < KW; kw++) {
        const int64_t k = 32 * (wb0 + kw) + t;
        const uint32_t x = (k < K && jw < nwb) ? B[k * ldb + jw] : 0u;
        out[kw] = transpose_bits<0>(0u, x);
    }
    uint32_t *dst = BT + (64 * c + lane) * ldbt + wb0;
    if constexpr (KW == 4)
        *reinterpret_cast<uint4 *>(dst) = uint4{out[0], out[1], out[2], out[3]};
    else
#pragma unroll
        for (int kw = 0; kw < KW; kw++) dst[kw] = out[kw];
}

// Closure update on the matrix cores: T_ij (|)= T_iK * T_Kj over a BRect
// (64-row chunks [r_lo, r_hi) minus [r_ex0, r_ex1), 32-bit words [w0a, w0b)
// and [w1a, w1b)) for the pivot block K = [k0, k0 + bs), in tiles of 64 rows
// x BJ words; PT is the transposed pivot-row panel (row j = column j of rows
// k0 .. k0 + bs - 1, 8 words, zero past bs and past column D).  Workgroup:
// four waves on four row chunks of one column chunk.
//
// Workgroup n of a launch runs on XCD n % 8 (the dispatcher's round robin).
// The workgroups are renumbered so that each XCD takes one contiguous range
// of the logical order, in which the column chunks of a row band come one
// after another: a wave's C rows are 8 bytes of a 128-byte line that the
// neighbouring column chunks also read and write, and those then meet in one
// L2 instead of moving the line through every XCD's L2.
__device__ __forceinline__ int xcd_contiguous(int n, int total) {
    const int x = n & 7, i = n >> 3;
    const int per = total >> 3, rem = total & 7;
    return x * per + min(x, rem) + i;
}

template <int F, int BJ>
__global__ void __launch_bounds__(256)
k_bool_fw_update_mfma(uint32_t *T, int64_t ld, int D, int k0, BRect q, int nch0, int nch,
                      const uint32_t *PT, int64_t ldpt) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lg = xcd_contiguous((int)blockIdx.x, (int)gridDim.x);
    const int band = lg / nch, cx = lg % nch;
    int rc = q.r_lo + band * 4 + wave;
    if (rc >= q.r_ex0) rc += q.r_ex1 - q.r_ex0;
    if (rc >= q.r_hi) return;
    const int w0 = cx < nch0 ? q.w0a + cx * BJ : q.w1a + (cx - nch0) * BJ;
    const int wend = cx < nch0 ? q.w0b : q.w1b;
    const int64_t row0 = (int64_t)rc * 64;
    const int nrows = (int)min<int64_t>(64, (int64_t)D - row0);
    const int kw0 = k0 >> 5;
    mfma_tile<F, BJ>(T + row0 * ld + w0, ld, T + row0 * ld + kw0, ld, ld - kw0,
                     PT + 32 * (int64_t)w0 * ldpt, ldpt, 1, nrows, min(BJ, wend - w0), true);
}

// Operand format of the matrix-core path: F4 unless the environment sets
// SR_MFMA_FORMAT=i8 (read at every launch, for comparison runs and tests).
int mfma_format() {
    const char *v = getenv("SR_MFMA_FORMAT");
    return (v && strcmp(v, "i8") == 0) ? kI8 : kF4;
}

constexpr int kMulBJ = 2;

// BT := the bit transpose of K x (32 nwb) B into n_rows_bt rows of 8 ngroups
// words; one word per wave while the grid is small (a round's pivot rows),
// four for large ones (a product's B).
hipError_t transpose(uint32_t *BT, int64_t ldbt, int64_t n_rows_bt, int ngroups, const uint32_t *B,
                     int64_t ldb, int64_t K, int64_t nwb, hipStream_t st) {
    const unsigned gx = (unsigned)((n_rows_bt / 64 + 3) / 4);
    if ((int64_t)gx * ngroups * 8 <= 4096)
        hipLaunchKernelGGL(k_bit_transpose<1>, dim3(gx, (unsigned)(8 * ngroups)), dim3(256), 0, st,
                           BT, ldbt, B, ldb, K, nwb, n_rows_bt);
    else
        hipLaunchKernelGGL(k_bit_transpose<4>, dim3(gx, (unsigned)(2 * ngroups)), dim3(256), 0, st,
                           BT, ldbt, B, ldb, K, nwb, n_rows_bt);
    return hipGetLastError();
}

}  // namespace

// BT of the product: rows = N rounded up to the column tile (plus nothing
// else), 8-word groups covering K.
size_t bool_mfma_work_bytes(int64_t R, int64_t K, int64_t N) {
    (void)R;
    const int64_t ngroups = (K + 255) / 256;
    const int64_t nrows = (N + 127) / 128 * 128;
    return (size_t)(nrows * ngroups * 8) * 4;
}

hipError_t launch_bool_mul_mfma(uint64_t *C, int64_t ldc, const uint64_t *A, int64_t lda,
                                const uint64_t *B, int64_t ldb, int64_t R, int64_t K, int64_t N,
                                bool accumulate, void *work, hipStream_t st) {
    // K = 0: the product is the zero matrix; hand it to the bit-sliced
    // kernels (which write the zeros, or leave C as it is)
    if (K == 0)
        return launch_bool_mul(C, ldc, A, lda, B, ldb, R, K, N, accumulate, kBoolPathBitwise, st);
    const int ngroups = (int)((K + 255) / 256);
    const int64_t nrows_bt = (N + 127) / 128 * 128;
    const int64_t ldbt = 8 * (int64_t)ngroups;
    uint32_t *BT = static_cast<uint32_t *>(work);
    const uint32_t *a = reinterpret_cast<const uint32_t *>(A);
    const uint32_t *b = reinterpret_cast<const uint32_t *>(B);
    const int64_t nwords = (N + 31) / 32;
    hipError_t e = transpose(BT, ldbt, nrows_bt, ngroups, b, 2 * ldb, K, nwords, st);
    if (e != hipSuccess) return e;
    const dim3 grid((unsigned)((nwords + kMulBJ - 1) / kMulBJ), (unsigned)((R + 255) / 256));
    uint32_t *c = reinterpret_cast<uint32_t *>(C);
    if (mfma_format() == kI8)
        hipLaunchKernelGGL((k_bool_mul_mfma<kI8, kMulBJ>), grid, dim3(256), 0, st, c, 2 * ldc, a,
                           2 * lda, 2 * lda, BT, ldbt, ngroups, R, nwords, accumulate ? 1 : 0);
    else
        hipLaunchKernelGGL((k_bool_mul_mfma<kF4, kMulBJ>), grid, dim3(256), 0, st, c, 2 * ldc, a,
                           2 * lda, 2 * lda, BT, ldbt, ngroups, R, nwords, accumulate ? 1 : 0);
    return hipGetLastError();
}

size_t bool_mfma_closure_work_bytes(int64_t D) {
    // two PT buffers (consecutive rounds), rows for every column word, 8
    // words each
    return 2 * (size_t)(((D + 31) / 32 + 4) * 32) * 32;
}

hipError_t launch_bool_pivot_transpose(uint32_t *PT, const uint32_t *T, int64_t ld, int64_t D,
                                       int k0, int bs, hipStream_t st) {
    const int64_t nwd = (D + 31) / 32;
    const int64_t nrows_pt = (nwd + 4) / 2 * 64;  // whole pairs of words, one pair spare
    return transpose(PT, 8, nrows_pt, 1, T + (int64_t)k0 * ld, ld, bs, nwd, st);
}

hipError_t launch_bool_fw_update_mfma(uint32_t *T, int64_t ld, int64_t D, int k0,
                                      const BRect &q, const uint32_t *PT, hipStream_t st) {
    constexpr int BJ = 2;
    const int nch0 = q.w0b > q.w0a ? (q.w0b - q.w0a + BJ - 1) / BJ : 0;
    const int nch1 = q.w1b > q.w1a ? (q.w1b - q.w1a + BJ - 1) / BJ : 0;
    const int nrows = (q.r_hi - q.r_lo) - (q.r_ex1 - q.r_ex0);
    if (nch0 + nch1 == 0 || nrows <= 0) return hipSuccess;
    const int nch = nch0 + nch1;
    const dim3 grid((unsigned)(nch * ((nrows + 3) / 4)));
    if (mfma_format() == kI8)
        hipLaunchKernelGGL((k_bool_fw_update_mfma<kI8, BJ>), grid, dim3(256), 0, st, T, ld, (int)D,
                           k0, q, nch0, nch, PT, (int64_t)8);
    else
        hipLaunchKernelGGL((k_bool_fw_update_mfma<kF4, BJ>), grid, dim3(256), 0, st, T, ld, (int)D,
                           k0, q, nch0, nch, PT, (int64_t)8);
    return hipGetLastError();
}

}  // namespace sr
