// Anti-distance semiring with 32-bit entries, S = 2^32 - 1 (the integer
// scaling of Sec. IV with 32-bit storage).  S - a is the bitwise complement,
// so a (x) b = max(a + b - S, 0) = b -sat (S - a) is one v_sub_u32 with clamp
// and (+) is v_max_u32; the products of two inner steps enter the accumulator
// through one v_max3_u32, so an update costs 1.5 VALU lane-operations (the
// 16-bit kernels do two updates per pair of packed operations).
//
// Same algorithms and schedule as the 16-bit path (Sec. II product and
// blocked Warshall/Floyd closure in rounds of 128 pivots: pivot tile, panels,
// update, with the next round's pivot and panels run beside the bulk of the
// current update on a second stream), with 32-bit wave tiles: a wavefront
// owns 64 rows (lane = row) x CW columns, the B row of each inner step is read
// with scalar loads and enters every instruction as its SGPR operand, and each
// lane reads its own row of A in 64-byte groups, one group ahead.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdlib.h>

#include <algorithm>

#include "sr_batch_dev.h"
#include "sr_internal.h"
#include "sr_tiles.h"  // kconst (scalar reads of B rows), Rect, panel_wgs

namespace sr {
namespace {

using dev::Rect;

constexpr int kUpdCW = 32;  // columns per wave tile: update and product
constexpr int kPanCW = 32;  // columns per wave tile: panels (the chunking of panel_wgs)
constexpr int kRW = 64;     // rows per wave tile

__device__ __forceinline__ uint32_t step32(uint32_t acc, uint32_t b, uint32_t na) {
    return __builtin_elementwise_max(acc, __builtin_elementwise_sub_sat(b, na));
}

// Two inner steps: max(acc, b0 -sat na0, b1 -sat na1), which the compiler
// emits as two v_sub_u32 (clamp) and one v_max3_u32.
__device__ __forceinline__ uint32_t step32x2(uint32_t acc, uint32_t b0, uint32_t na0, uint32_t b1,
                                             uint32_t na1) {
    return __builtin_elementwise_max(
        __builtin_elementwise_max(acc, __builtin_elementwise_sub_sat(b0, na0)),
        __builtin_elementwise_sub_sat(b1, na1));
}

// ---------------------------------------------------------------------------
// One wavefront: C (+)= A * B (or C := A * B) for rows [0, nrows), lane = row,
// and columns [0, ncols), over K inner steps.  The caller guarantees that CW
// columns of every B row are readable from B (ncols may be less: the extra
// columns feed accumulators that are not stored).  FULLC: ncols == CW (whole
// 16-byte C accesses); else C is read and written entry by entry.  Rows >=
// nrows compute on row 0 and store nothing.  A, B and C rows are 16-byte
// aligned.  With sync, a workgroup barrier separates every read of the tile's
// operands from its stores (the whole workgroup must call this).
// ---------------------------------------------------------------------------
template <int CW, bool FULLC>
__device__ __forceinline__ void tile32_body(uint32_t *C, int64_t ldc, const uint32_t *A,
                                            int64_t lda, const uint32_t *B, int64_t ldb,
                                            int nrows, int ncols, int K, bool accumulate,
                                            bool sync) {
    static_assert(CW % 4 == 0 && CW <= 64, "CW: multiple of 4, at most 64");
    constexpr int KU = 64 / CW;  // B rows per batch of scalar loads (64 SGPRs)
    constexpr int AG = 16;       // A entries per lane per group (64 bytes)
    const int lane = threadIdx.x & 63;
    const bool live = lane < nrows;
    const int64_t r = live ? lane : 0;
    uint32_t *crow = C + r * ldc;
    uint32_t acc[CW];
    if (accumulate && FULLC) {
#pragma unroll
        for (int q = 0; q < CW / 4; q++) {
            const uint4 v = reinterpret_cast<const uint4 *>(crow)[q];
            acc[4 * q] = v.x;
            acc[4 * q + 1] = v.y;
            acc[4 * q + 2] = v.z;
            acc[4 * q + 3] = v.w;
        }
    } else {
#pragma unroll
        for (int w = 0; w < CW; w++) acc[w] = (accumulate && w < ncols) ? crow[w] : 0u;
    }

    const uint32_t *arow = A + r * lda;
    int k = 0;
    if (K >= AG) {
        uint4 anext[AG / 4];
#pragma unroll
        for (int q = 0; q < AG / 4; q++) anext[q] = reinterpret_cast<const uint4 *>(arow)[q];
        for (; k + AG <= K; k += AG) {
            uint32_t na[AG];
#pragma unroll
            for (int q = 0; q < AG / 4; q++) {
                na[4 * q] = ~anext[q].x;
                na[4 * q + 1] = ~anext[q].y;
                na[4 * q + 2] = ~anext[q].z;
                na[4 * q + 3] = ~anext[q].w;
            }
            // issue the next group's loads only after the complements above
            // have consumed this group (the empty asm statements emit
            // nothing: they pin each value, then order the loads after them),
            // so the loads reuse its registers
#pragma unroll
            for (int i = 0; i < AG; i++) asm volatile("" : "+v"(na[i]));
            asm volatile("" ::: "memory");
            if (k + 2 * AG <= K) {
#pragma unroll
                for (int q = 0; q < AG / 4; q++)
                    anext[q] = reinterpret_cast<const uint4 *>(arow + k + AG)[q];
            }
#pragma unroll
            for (int kg = 0; kg < AG; kg += KU) {
                // two inner steps per accumulator update: the (+) of the
                // accumulator with both products is one v_max3_u32, so a
                // pair of updates costs three lane-operations instead of four
                // this group's B rows, loaded before its updates (one wait
                // per group, as in the 16-bit tiles)
                uint32_t bg[KU][CW];
#pragma unroll
                for (int kk = 0; kk < KU; kk++) {
                    const kconst uint32_t *bp =
                        (const kconst uint32_t *)(B + (int64_t)(k + kg + kk) * ldb);
#pragma unroll
                    for (int w = 0; w < CW; w++) bg[kk][w] = bp[w];
                }
#pragma unroll
                for (int kk = 0; kk < KU; kk += 2) {
#pragma unroll
                    for (int w = 0; w < CW; w++)
                        acc[w] = step32x2(acc[w], bg[kk][w], na[kg + kk], bg[kk + 1][w],
                                          na[kg + kk + 1]);
                }
            }
        }
    }
    for (; k < K; k++) {
        const uint32_t na = ~arow[k];
        const kconst uint32_t *brow = (const kconst uint32_t *)(B + (int64_t)k * ldb);
#pragma unroll
        for (int w = 0; w < CW; w++) acc[w] = step32(acc[w], brow[w], na);
    }

    if (sync) __syncthreads();
    if (!live) return;
    if (FULLC) {
#pragma unroll
        for (int q = 0; q < CW / 4; q++)
            reinterpret_cast<uint4 *>(crow)[q] =
                uint4{acc[4 * q], acc[4 * q + 1], acc[4 * q + 2], acc[4 * q + 3]};
    } else {
#pragma unroll
        for (int w = 0; w < CW; w++)
            if (w < ncols) crow[w] = acc[w];
    }
}

// A tile of nrows x ncols at C (ncols <= CW).  bspan: entries of each B row
// readable from B.  When a whole CW-column segment fits the tile runs as one;
// otherwise (the last columns of a row whose padded length is not a multiple
// of CW) as 4-column tiles, whose 16-byte segments always fit because rows
// are padded to 16 bytes.  With sync the whole workgroup must call this (it
// executes one barrier, after the stores of the 4-column tiles in that case;
// a panel update stays exact under that order because the pivot tile is
// closed: any mix of old and new operand entries gives the same result).
template <int CW>
__device__ __forceinline__ void tile32(uint32_t *C, int64_t ldc, const uint32_t *A, int64_t lda,
                                       const uint32_t *B, int64_t ldb, int nrows, int ncols,
                                       int64_t bspan, int K, bool accumulate, bool sync) {
    if (nrows <= 0 || ncols <= 0) {
        if (sync) __syncthreads();
        return;
    }
    if (bspan >= CW) {
        if (ncols >= CW)
            tile32_body<CW, true>(C, ldc, A, lda, B, ldb, nrows, CW, K, accumulate, sync);
        else
            tile32_body<CW, false>(C, ldc, A, lda, B, ldb, nrows, ncols, K, accumulate, sync);
        return;
    }
    for (int c = 0; c < ncols; c += 4)
        tile32_body<4, false>(C + c, ldc, A, lda, B + c, ldb, nrows, min(4, ncols - c), K,
                              accumulate, false);
    if (sync) __syncthreads();
}

// ---------------------------------------------------------------------------
// Product: grid (column chunks, row groups of 4 waves); the four waves of a
// workgroup are stacked along the rows and share the column chunk.  FULL:
// every chunk of the launch has CW columns inside N (a partial last chunk is
// a separate FULL = false launch).  col_base: first column of chunk 0; bmax:
// entries of each B row readable from B.
// ---------------------------------------------------------------------------
template <int CW, bool FULL>
__global__ void __launch_bounds__(256)
k_ad32_mul(uint32_t *C, int64_t ldc, const uint32_t *A, int64_t lda, const uint32_t *B,
           int64_t ldb, int64_t R, int K, int64_t N, int64_t col_base, int accumulate,
           int64_t bmax, const int *gate, const uint32_t *prev, int *flag) {
    if (gate && *gate == 0) return;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t row0 = ((int64_t)blockIdx.y * 4 + wave) * kRW;
    const int64_t col0 = col_base + (int64_t)blockIdx.x * CW;
    if (row0 >= R) return;
    const int nrows = (int)min<int64_t>(kRW, R - row0);
    const int ncols = FULL ? CW : (int)min<int64_t>(CW, N - col0);
    if (FULL)
        tile32_body<CW, true>(C + row0 * ldc + col0, ldc, A + row0 * lda, lda, B + col0, ldb,
                              nrows, CW, K, accumulate != 0, false);
    else
        tile32<CW>(C + row0 * ldc + col0, ldc, A + row0 * lda, lda, B + col0, ldb, nrows, ncols,
                   bmax - col0, K, accumulate != 0, false);
    if (prev) {
        // change check: this lane's row of the tile just stored, read back,
        // against the same entries of prev (same layout as C)
        const int lane = threadIdx.x & 63;
        bool diff = false;
        if (lane < nrows) {
            const uint32_t *c = C + (row0 + lane) * ldc + col0;
            const uint32_t *p = prev + (row0 + lane) * ldc + col0;
            for (int j = 0; j < ncols; j++) diff |= c[j] != p[j];
        }
        if (__any(diff) && lane == 0) *flag = 1;
    }
}

// Product with the inner dimension split over the KS waves of a workgroup,
// for products with too few output tiles to fill the chip (the K-split
// kernel of the 16-bit path, with 32-bit tiles): all KS waves take the same
// 64-row x CW-column tile of C (every chunk of the launch has CW columns
// inside N), wave w the inner steps [w kq, (w + 1) kq) (kq a multiple of 32);
// their partial results meet in LDS, where the (+) of the KS partials (and of
// C when accumulating) is taken.  (+) is max, so splitting the inner loop
// changes nothing in the result.  With prev, each stored word is compared
// with prev's (the squaring's change flag).
template <int CW, int KS>
__device__ __forceinline__ void ksplit32_tile(uint32_t (*part)[kRW][CW], uint32_t *C, int64_t ldc,
                                              const uint32_t *A, int64_t lda, const uint32_t *B,
                                              int64_t ldb, int64_t R, int K, int kq,
                                              int accumulate, const uint32_t *prev, int *flag,
                                              int64_t row0, int64_t col0) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nrows = (int)min<int64_t>(kRW, R - row0);
    const int k0 = min(K, wave * kq), k1 = min(K, k0 + kq);
    // this wave's partial product (rows >= nrows are not written)
    tile32_body<CW, true>(&part[wave][0][0], CW, A + row0 * lda + k0, lda,
                          B + (int64_t)k0 * ldb + col0, ldb, nrows, CW, k1 - k0, false, false);
    __syncthreads();
    bool diff = false;
    for (int wi = threadIdx.x; wi < kRW * CW; wi += 64 * KS) {
        const int row = wi / CW, col = wi % CW;
        if (row >= nrows) continue;
        uint32_t v = part[0][row][col];
#pragma unroll
        for (int q = 1; q < KS; q++) v = max(v, part[q][row][col]);
        uint32_t *dst = C + (row0 + row) * ldc + col0 + col;
        if (accumulate) v = max(v, *dst);
        *dst = v;
        if (prev) diff |= v != prev[(row0 + row) * ldc + col0 + col];
    }
    if (prev && __any(diff) && (threadIdx.x & 63) == 0) *flag = 1;
}

template <int CW, int KS>
__global__ void __launch_bounds__(64 * KS)
k_ad32_mul_ksplit(uint32_t *C, int64_t ldc, const uint32_t *A, int64_t lda, const uint32_t *B,
                  int64_t ldb, int64_t R, int K, int kq, int accumulate, const int *gate,
                  const uint32_t *prev, int *flag) {
    __shared__ uint32_t part[KS][kRW][CW];
    if (gate && *gate == 0) return;  // (uniform over the workgroup: before any barrier)
    ksplit32_tile<CW, KS>(part, C, ldc, A, lda, B, ldb, R, K, kq, accumulate, prev, flag,
                          (int64_t)blockIdx.y * kRW, (int64_t)blockIdx.x * CW);
}

// Up to four independent products in one launch of the K-split tiles (the
// blocks of a big-block round; the 16-bit path's k_ad_mul_ksplit_group with
// 32-bit tiles): workgroups [end_{q-1}, end_q) take the nx_q x ny_q tiles of
// product q, row-major.
struct Ksplit32Problem {
    uint32_t *C;
    const uint32_t *A, *B;
    int64_t ldc, lda, ldb, R;
    int K, kq, nx, end;
};
struct Ksplit32Group {
    Ksplit32Problem p[4];
    int n, accumulate;
};

template <int CW, int KS>
__global__ void __launch_bounds__(64 * KS) k_ad32_mul_ksplit_group(Ksplit32Group g) {
    __shared__ uint32_t part[KS][kRW][CW];
    const int b = blockIdx.x;
    int q = 0;
    while (q + 1 < g.n && b >= g.p[q].end) q++;
    const Ksplit32Problem &p = g.p[q];
    const int local = b - (q > 0 ? g.p[q - 1].end : 0);
    ksplit32_tile<CW, KS>(part, p.C, p.ldc, p.A, p.lda, p.B, p.ldb, p.R, p.K, p.kq, g.accumulate,
                          nullptr, nullptr, (int64_t)(local / p.nx) * kRW,
                          (int64_t)(local % p.nx) * CW);
}

// ---------------------------------------------------------------------------
// Pivot tile: Warshall closure of the bs x bs tile at T (bs <= 128) by one
// 256-thread workgroup.  Thread (ty, tx) = (t / 16, t % 16) holds rows
// 8ty..8ty+7 x columns 8tx..8tx+7 in registers.  Row k and column k do not
// change during step k (T_kk (x) x <= x since T_kk <= S), so the owners of
// row k and column k publish them in LDS (the column as S - value), one
// barrier per step, two buffers alternating so that step k+1's publication
// cannot overwrite what a slower thread still reads for step k.  Entries
// outside bs x bs are held as 0, the additive zero, and stay 0.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void pivot32_tile(uint32_t *T, int64_t ld, int bs, uint32_t *lds_row,
                                             uint32_t *lds_col) {
    const int t = threadIdx.x;
    const int tx = t & 15, ty = t >> 4;
    const int c0 = 8 * tx;
    uint32_t acc[8][8];
#pragma unroll
    for (int i = 0; i < 8; i++) {
        const int row = 8 * ty + i;
        const uint32_t *src = T + (int64_t)row * ld + c0;
        if (row < bs && c0 + 8 <= bs) {
            const uint4 v0 = reinterpret_cast<const uint4 *>(src)[0];
            const uint4 v1 = reinterpret_cast<const uint4 *>(src)[1];
            acc[i][0] = v0.x, acc[i][1] = v0.y, acc[i][2] = v0.z, acc[i][3] = v0.w;
            acc[i][4] = v1.x, acc[i][5] = v1.y, acc[i][6] = v1.z, acc[i][7] = v1.w;
        } else {
#pragma unroll
            for (int c = 0; c < 8; c++) acc[i][c] = (row < bs && c0 + c < bs) ? src[c] : 0u;
        }
    }

    const int nq = (bs + 7) >> 3;
    for (int q = 0; q < nq; q++) {
#pragma unroll
        for (int s = 0; s < 8; s++) {
            uint32_t *rb = lds_row + (s & 1) * 128;
            uint32_t *cb = lds_col + (s & 1) * 128;
            if (ty == q) {
                reinterpret_cast<uint4 *>(rb)[2 * tx] =
                    uint4{acc[s][0], acc[s][1], acc[s][2], acc[s][3]};
                reinterpret_cast<uint4 *>(rb)[2 * tx + 1] =
                    uint4{acc[s][4], acc[s][5], acc[s][6], acc[s][7]};
            }
            if (tx == q) {
                reinterpret_cast<uint4 *>(cb)[2 * ty] =
                    uint4{~acc[0][s], ~acc[1][s], ~acc[2][s], ~acc[3][s]};
                reinterpret_cast<uint4 *>(cb)[2 * ty + 1] =
                    uint4{~acc[4][s], ~acc[5][s], ~acc[6][s], ~acc[7][s]};
            }
            __syncthreads();
            const uint4 b0 = reinterpret_cast<const uint4 *>(rb)[2 * tx];
            const uint4 b1 = reinterpret_cast<const uint4 *>(rb)[2 * tx + 1];
            const uint4 n0 = reinterpret_cast<const uint4 *>(cb)[2 * ty];
            const uint4 n1 = reinterpret_cast<const uint4 *>(cb)[2 * ty + 1];
            const uint32_t b[8] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w};
            const uint32_t nn[8] = {n0.x, n0.y, n0.z, n0.w, n1.x, n1.y, n1.z, n1.w};
#pragma unroll
            for (int i = 0; i < 8; i++)
#pragma unroll
                for (int c = 0; c < 8; c++) acc[i][c] = step32(acc[i][c], b[c], nn[i]);
        }
    }

#pragma unroll
    for (int i = 0; i < 8; i++) {
        const int row = 8 * ty + i;
        if (row >= bs || c0 >= bs) continue;
        uint32_t *dst = T + (int64_t)row * ld + c0;
        if (c0 + 8 <= bs) {
            reinterpret_cast<uint4 *>(dst)[0] = uint4{acc[i][0], acc[i][1], acc[i][2], acc[i][3]};
            reinterpret_cast<uint4 *>(dst)[1] = uint4{acc[i][4], acc[i][5], acc[i][6], acc[i][7]};
        } else {
#pragma unroll
            for (int c = 0; c < 8; c++)
                if (c0 + c < bs) dst[c] = acc[i][c];
        }
    }
}

__global__ void __launch_bounds__(256) k_ad32_pivot(uint32_t *T, int64_t ld, int bs, int prio) {
    if (prio) __builtin_amdgcn_s_setprio(2);
    __shared__ uint32_t lds_row[2 * 128];
    __shared__ uint32_t lds_col[2 * 128];
    pivot32_tile(T, ld, bs, lds_row, lds_col);
}

// ---------------------------------------------------------------------------
// Panels of round K = [k0, k0 + bs), one workgroup (id bid).  Workgroups
// [0, n_rowwg) take the row panel T_Kj (+)= T_KK * T_Kj: two 64-row halves of
// the pivot rows times two 32-column chunks outside the pivot block.  The
// rest take the column panel T_iK (+)= T_iK * T_KK: one 64-row chunk outside
// the pivot block times the four 32-column chunks of the pivot block.  Each
// panel tile is written by one workgroup, after a barrier that follows every
// read of the workgroup's operands.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void panels32_wg(uint32_t *T, int64_t ld, int D, int k0, int bs,
                                            int n_rowwg, int bid) {
    constexpr int CW = kPanCW;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (bid < n_rowwg) {
        const int kc0 = k0 / CW, kc1 = (k0 + bs + CW - 1) / CW;
        const int cc = 2 * bid + (wave >> 1);
        const int c = cc < kc0 ? cc : cc + (kc1 - kc0);
        const int64_t col0 = (int64_t)c * CW;
        const int rofs = (wave & 1) * 64;
        const int nrows = min(64, bs - rofs);
        const int ncols = (int)min<int64_t>(CW, (int64_t)D - col0);
        const int64_t r0 = (int64_t)k0 + rofs;
        tile32<CW>(T + r0 * ld + col0, ld, T + r0 * ld + k0, ld, T + (int64_t)k0 * ld + col0, ld,
                   nrows, ncols, ld - col0, bs, true, true);
    } else {
        const int kr0 = k0 / 64, kr1 = (k0 + bs + 63) / 64;
        const int rc = bid - n_rowwg;
        const int rchunk = rc < kr0 ? rc : rc + (kr1 - kr0);
        const int64_t row0 = (int64_t)rchunk * 64;
        const int nrows = (int)min<int64_t>(64, (int64_t)D - row0);
        const int cofs = wave * CW;
        const int ncols = min(CW, bs - cofs);
        tile32<CW>(T + row0 * ld + k0 + cofs, ld, T + row0 * ld + k0, ld,
                   T + (int64_t)k0 * ld + k0 + cofs, ld, nrows, ncols, ld - k0 - cofs, bs, true,
                   true);
    }
}

__global__ void __launch_bounds__(256)
k_ad32_panels(uint32_t *T, int64_t ld, int D, int k0, int bs, int n_rowwg, int prio) {
    if (prio) __builtin_amdgcn_s_setprio(2);
    panels32_wg(T, ld, D, k0, bs, n_rowwg, (int)blockIdx.x);
}

// ---------------------------------------------------------------------------
// Update of round K over a rectangle of tiles: row chunks (64 rows)
// [r_lo, r_hi) minus [r_ex0, r_ex1), column chunks (CW columns) [c_lo, c_hi)
// minus [c_ex0, c_ex1); T_ij (+)= T_iK * T_Kj.  Workgroup (bx, by): column
// chunk bx of the selection, row chunks 4 by .. 4 by + 3 (one per wave).
// FULL: every selected column chunk lies inside D.
// ---------------------------------------------------------------------------
template <int CW, bool FULL>
__global__ void __launch_bounds__(256)
k_ad32_update(uint32_t *T, int64_t ld, int D, int k0, int bs, Rect q, int prio) {
    if (prio) __builtin_amdgcn_s_setprio(2);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int c = q.c_lo + (int)blockIdx.x;
    if (c >= q.c_ex0) c += q.c_ex1 - q.c_ex0;
    int rc = q.r_lo + (int)blockIdx.y * 4 + wave;
    if (rc >= q.r_ex0) rc += q.r_ex1 - q.r_ex0;
    if (rc >= q.r_hi || c >= q.c_hi) return;
    const int64_t row0 = (int64_t)rc * kRW, col0 = (int64_t)c * CW;
    const int nrows = (int)min<int64_t>(kRW, (int64_t)D - row0);
    uint32_t *dst = T + row0 * ld + col0;
    const uint32_t *a = T + row0 * ld + k0;
    const uint32_t *b = T + (int64_t)k0 * ld + col0;
    if (FULL)
        tile32_body<CW, true>(dst, ld, a, ld, b, ld, nrows, CW, bs, true, false);
    else
        tile32<CW>(dst, ld, a, ld, b, ld, nrows, (int)min<int64_t>(CW, (int64_t)D - col0),
                   ld - col0, bs, true, false);
}

// ---------------------------------------------------------------------------
// Batched closures of 32-bit matrices: the launches of the batched closure
// (sr_batched.hip: work lists, XCD-aware order) with the 32-bit workgroup
// bodies above.  Update tiles are 64 rows x kUpdCW columns, the geometry of
// the plan's update-tile code 2; the panels use panel_wgs' geometry, as the
// single-matrix panels do.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k_batch32_pivot(const BatchDesc *desc, const BatchItem *items, int kb) {
    __shared__ uint32_t lds_row[2 * 128];
    __shared__ uint32_t lds_col[2 * 128];
    const BatchDesc d = bdev::cdesc(desc, bdev::citems(items)[blockIdx.x].graph);
    const int k0 = kb * kAdBlock, bs = min(kAdBlock, d.D - k0);
    pivot32_tile(d.T32 + (int64_t)k0 * d.ld + k0, d.ld, bs, lds_row, lds_col);
}

__global__ void __launch_bounds__(256)
k_batch32_panels(const BatchDesc *desc, const BatchItem *items, int n_items, int kb, int xmap) {
    const int bid = xmap ? bdev::xcd_order((int)blockIdx.x, (int)gridDim.x, xmap) : (int)blockIdx.x;
    const int i = bdev::find_item(items, n_items, bid);
    const BatchDesc d = bdev::cdesc(desc, bdev::citems(items)[i].graph);
    const int k0 = kb * kAdBlock, bs = min(kAdBlock, d.D - k0);
    int n_rowwg = 0, n_colwg = 0;
    dev::panel_wgs(d.D, k0, bs, &n_rowwg, &n_colwg);
    panels32_wg(d.T32, d.ld, d.D, k0, bs, n_rowwg, bid - bdev::citems(items)[i].first);
}

__global__ void __launch_bounds__(256)
k_batch32_update(const BatchDesc *desc, const BatchItem *items, int n_items, int kb, int n_waves,
                 int xmap) {
    const int bid = xmap ? bdev::xcd_order((int)blockIdx.x, (int)gridDim.x, xmap) : (int)blockIdx.x;
    const int gw = bid * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (gw >= n_waves) return;
    const int i = bdev::find_item(items, n_items, gw);
    const BatchDesc d = bdev::cdesc(desc, bdev::citems(items)[i].graph);
    const int k0 = kb * kAdBlock, bs = min(kAdBlock, d.D - k0);
    int nc = 0, nr = 0;
    const Rect q = bdev::update_rect(d.D, kb, kRW, kUpdCW, &nc, &nr);
    const int local = gw - bdev::citems(items)[i].first;
    // column-chunk major, as the 16-bit batch
    int c = local / nr, rc = local % nr;
    if (c >= q.c_ex0) c += q.c_ex1 - q.c_ex0;
    if (rc >= q.r_ex0) rc += q.r_ex1 - q.r_ex0;
    if (rc >= q.r_hi || c >= q.c_hi) return;
    const int64_t row0 = (int64_t)rc * kRW, col0 = (int64_t)c * kUpdCW;
    const int nrows = (int)min<int64_t>(kRW, (int64_t)d.D - row0);
    uint32_t *dst = d.T32 + row0 * d.ld + col0;
    const uint32_t *a = d.T32 + row0 * d.ld + k0;
    const uint32_t *b = d.T32 + (int64_t)k0 * d.ld + col0;
    if (col0 + kUpdCW <= d.D)
        tile32_body<kUpdCW, true>(dst, d.ld, a, d.ld, b, d.ld, nrows, kUpdCW, bs, true, false);
    else
        tile32<kUpdCW>(dst, d.ld, a, d.ld, b, d.ld, nrows, (int)min<int64_t>(kUpdCW, d.D - col0),
                       d.ld - col0, bs, true, false);
}

// Entries of every graph complemented in place (S - a), rows [32 y, 32 y +
// 32) of graph blockIdx.x; and the diagonal of every graph := value.
__global__ void __launch_bounds__(256) k_batch32_not(const BatchDesc *desc) {
    const BatchDesc d = desc[blockIdx.x];
    const int64_t r0 = (int64_t)blockIdx.y * 32;
    if (r0 >= d.D) return;
    const int64_t nr = min<int64_t>(32, (int64_t)d.D - r0);
    for (int64_t g = threadIdx.x; g < nr * d.D; g += 256) {
        uint32_t *e = d.T32 + (r0 + g / d.D) * d.ld + (g % d.D);
        *e = ~*e;
    }
}

__global__ void __launch_bounds__(256) k_batch32_diag(const BatchDesc *desc, uint32_t value) {
    const BatchDesc d = desc[blockIdx.x];
    for (int64_t i = threadIdx.x; i < d.D; i += 256) d.T32[i * d.ld + i] = value;
}

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------
template <int CW>
hipError_t mul_cw(uint32_t *C, int64_t ldc, const uint32_t *A, int64_t lda, const uint32_t *B,
                  int64_t ldb, int64_t R, int64_t K, int64_t N, bool acc, int64_t bmax,
                  const int *gate, const uint32_t *prev, int *flag, hipStream_t st) {
    const unsigned gy = (unsigned)((R + 4 * kRW - 1) / (4 * kRW));
    const int64_t nfull = N / CW;
    if (nfull > 0) {
        hipLaunchKernelGGL((k_ad32_mul<CW, true>), dim3((unsigned)nfull, gy), dim3(256), 0, st, C,
                           ldc, A, lda, B, ldb, R, (int)K, N, (int64_t)0, acc ? 1 : 0, bmax,
                           gate, prev, flag);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (N % CW) {
        hipLaunchKernelGGL((k_ad32_mul<CW, false>), dim3(1u, gy), dim3(256), 0, st, C, ldc, A, lda,
                           B, ldb, R, (int)K, N, nfull * CW, acc ? 1 : 0, bmax, gate, prev,
                           flag);
        return hipGetLastError();
    }
    return hipSuccess;
}

int blocks_of(int64_t D) { return (int)((D + kAdBlock - 1) / kAdBlock); }
int block_k0(int64_t kb) { return (int)(kb * kAdBlock); }
int block_bs(int64_t D, int64_t kb) { return (int)std::min<int64_t>(kAdBlock, D - kb * kAdBlock); }

// chunks [lo, hi) of width w covering pivot block kb
void block_chunks(int64_t D, int64_t kb, int w, int *lo, int *hi) {
    const int k0 = block_k0(kb), bs = block_bs(D, kb);
    *lo = k0 / w;
    *hi = (k0 + bs + w - 1) / w;
}

// SR_PRIO=0 keeps the critical-path kernels at the default wave priority;
// SR_LOOKAHEAD=0 runs every round's phases in order on the caller's stream.
struct Tuning32 {
    bool prio = true, lookahead = true;
    Tuning32() {
        if (const char *v = getenv("SR_PRIO")) prio = atoi(v) != 0;
        if (const char *v = getenv("SR_LOOKAHEAD")) lookahead = atoi(v) != 0;
    }
};
const Tuning32 &tuning() {
    static const Tuning32 t;
    return t;
}

hipError_t update_launch(uint32_t *T, int64_t ld, int64_t D, int k0, int bs, const Rect &q,
                         bool full, int prio, hipStream_t st) {
    const int nr = (q.r_hi - q.r_lo) - (q.r_ex1 - q.r_ex0);
    const int nc = (q.c_hi - q.c_lo) - (q.c_ex1 - q.c_ex0);
    if (nr <= 0 || nc <= 0) return hipSuccess;
    const dim3 grid((unsigned)nc, (unsigned)((nr + 3) / 4));
    if (full)
        hipLaunchKernelGGL((k_ad32_update<kUpdCW, true>), grid, dim3(256), 0, st, T, ld, (int)D,
                           k0, bs, q, prio);
    else
        hipLaunchKernelGGL((k_ad32_update<kUpdCW, false>), grid, dim3(256), 0, st, T, ld, (int)D,
                           k0, bs, q, prio);
    return hipGetLastError();
}

// Update of round kb over a rectangle of tiles (64-row chunks x kUpdCW-column
// chunks, one excluded range of each; an empty range is moved to the end).
// The full column chunks go to the hot kernel; a partial last chunk of the
// matrix (D not a multiple of the chunk width), if selected, to the edge
// kernel.  critical: the launch is on the chain that the next round waits
// for, its waves run at a raised priority.
hipError_t update_rect(uint32_t *T, int64_t ld, int64_t D, int64_t kb, Rect q, double units,
                       bool critical, hipStream_t st) {
    if (q.r_ex1 <= q.r_ex0) q.r_ex0 = q.r_ex1 = q.r_hi;
    if (q.c_ex1 <= q.c_ex0) q.c_ex0 = q.c_ex1 = q.c_hi;
    const int k0 = block_k0(kb), bs = block_bs(D, kb);
    const int prio = critical && tuning().prio ? 1 : 0;
    const int last = (int)((D + kUpdCW - 1) / kUpdCW) - 1;
    const bool partial = (D % kUpdCW) != 0 && q.c_lo <= last && last < q.c_hi &&
                         !(q.c_ex0 <= last && last < q.c_ex1);
    Rect hot = q;
    if (partial) {
        // the last chunk is the final one of the range: drop it from the hot launch
        hot.c_hi = last;
        hot.c_ex0 = std::min(hot.c_ex0, hot.c_hi);
        hot.c_ex1 = std::min(hot.c_ex1, hot.c_hi);
    }
    const bool prof = prof_on();
    if (prof) prof_begin(st);
    hipError_t e = update_launch(T, ld, D, k0, bs, hot, true, prio, st);
    if (e == hipSuccess && partial) {
        const Rect edge{q.r_lo, q.r_hi, q.r_ex0, q.r_ex1, last, last + 1, last + 1, last + 1};
        e = update_launch(T, ld, D, k0, bs, edge, false, prio, st);
    }
    if (prof) prof_end(st, 1, 2, units);
    return e;
}

hipError_t pivot_round(uint32_t *T, int64_t ld, int64_t D, int64_t kb, hipStream_t st) {
    const int64_t k0 = block_k0(kb);
    const int bs = block_bs(D, kb);
    const bool prof = prof_on();
    if (prof) prof_begin(st);
    hipLaunchKernelGGL(k_ad32_pivot, dim3(1), dim3(256), 0, st, T + k0 * ld + k0, ld, bs,
                       tuning().prio ? 1 : 0);
    hipError_t e = hipGetLastError();
    if (prof) prof_end(st, 1, 0, (double)bs * bs * bs);
    return e;
}

hipError_t panels_round(uint32_t *T, int64_t ld, int64_t D, int64_t kb, hipStream_t st) {
    const int k0 = block_k0(kb), bs = block_bs(D, kb);
    int n_rowwg = 0, n_colwg = 0;
    dev::panel_wgs(D, k0, bs, &n_rowwg, &n_colwg);
    const int n = n_rowwg + n_colwg;
    if (n <= 0) return hipSuccess;
    const bool prof = prof_on();
    if (prof) prof_begin(st);
    hipLaunchKernelGGL(k_ad32_panels, dim3((unsigned)n), dim3(256), 0, st, T, ld, (int)D, k0, bs,
                       n_rowwg, tuning().prio ? 1 : 0);
    hipError_t e = hipGetLastError();
    if (prof) prof_end(st, 1, 1, 2.0 * (double)(D - bs) * bs * bs);
    return e;
}

// Closure driver.  Round kb: pivot(kb), panels(kb), update(kb).  With the
// second stream the update is split as in the 16-bit driver: A(kb), the
// tiles of row and column block kb+1 (outside block kb), runs on the caller's
// stream followed by pivot(kb+1) and panels(kb+1); B(kb), the rest, runs on
// the second stream, queued behind B(kb-1) as soon as panels(kb) is done.
// A(kb) writes tiles of row block kb+1 that B(kb-1) also writes, so the
// caller's stream waits for B(kb-1) before A(kb).  B(kb) reads only row and
// column block kb, which round kb+1 does not write.
hipError_t closure32(uint32_t *T, int64_t ld, int64_t D, bool serial, hipStream_t st,
                     bool aux_create) {
    const int nb = blocks_of(D);
    const int nrc = (int)((D + kRW - 1) / kRW), ncc = (int)((D + kUpdCW - 1) / kUpdCW);
    hipError_t e = pivot_round(T, ld, D, 0, st);
    if (e != hipSuccess || nb == 1) return e;
    if ((e = panels_round(T, ld, D, 0, st)) != hipSuccess) return e;
    Aux *aux = (nb > 2 && !serial && tuning().lookahead) ? aux_acquire(st, aux_create) : nullptr;
    for (int kb = 0; kb < nb; kb++) {
        int rl, rh, cl, ch;
        block_chunks(D, kb, kRW, &rl, &rh);
        block_chunks(D, kb, kUpdCW, &cl, &ch);
        const double bs = block_bs(D, kb);
        if (kb + 1 == nb || !aux) {
            if (aux && kb > 0) e = hipStreamWaitEvent(st, aux->ev_aux[(kb - 1) & 1], 0);
            const double rest = (double)D - bs;
            if (e == hipSuccess)
                e = update_rect(T, ld, D, kb, Rect{0, nrc, rl, rh, 0, ncc, cl, ch},
                                rest * rest * bs, false, st);
            if (e == hipSuccess && kb + 1 < nb) e = pivot_round(T, ld, D, kb + 1, st);
            if (e == hipSuccess && kb + 1 < nb) e = panels_round(T, ld, D, kb + 1, st);
            if (e != hipSuccess) break;
            continue;
        }
        int rl1, rh1, cl1, ch1;
        block_chunks(D, kb + 1, kRW, &rl1, &rh1);
        block_chunks(D, kb + 1, kUpdCW, &cl1, &ch1);
        const double bs1 = block_bs(D, kb + 1);
        const double rest2 = (double)D - bs - bs1;
        // B(kb) on the second stream, after panels(kb)
        e = hipEventRecord(aux->ev_main, st);
        if (e == hipSuccess) e = hipStreamWaitEvent(aux->stream, aux->ev_main, 0);
        if (e == hipSuccess)
            e = update_rect(T, ld, D, kb, Rect{0, nrc, rl, rh1, 0, ncc, cl, ch1},
                            rest2 * rest2 * bs, false, aux->stream);
        if (e == hipSuccess) e = hipEventRecord(aux->ev_aux[kb & 1], aux->stream);
        if (e == hipSuccess && kb > 0) e = hipStreamWaitEvent(st, aux->ev_aux[(kb - 1) & 1], 0);
        // A(kb): row block kb+1 (columns outside block kb), then column block
        // kb+1 (rows outside blocks kb and kb+1); then the next pivot and panels
        if (e == hipSuccess)
            e = update_rect(T, ld, D, kb, Rect{rl1, rh1, rh1, rh1, 0, ncc, cl, ch},
                            bs1 * ((double)D - bs) * bs, true, st);
        if (e == hipSuccess)
            e = update_rect(T, ld, D, kb, Rect{0, nrc, rl, rh1, cl1, ch1, ch1, ch1},
                            rest2 * bs1 * bs, true, st);
        if (e == hipSuccess) e = pivot_round(T, ld, D, kb + 1, st);
        if (e == hipSuccess) e = panels_round(T, ld, D, kb + 1, st);
        if (e != hipSuccess) break;
    }
    if (aux) aux_release(aux);
    return e;
}

}  // namespace

hipError_t launch_ad32_mul(uint32_t *C, int64_t ldc, const uint32_t *A, int64_t lda,
                           const uint32_t *B, int64_t ldb, int64_t R, int64_t K, int64_t N,
                           bool accumulate, hipStream_t stream, int64_t bspan,
                           const int *gate, const uint32_t *prev, int *flag) {
    const int64_t bmax = bspan >= 0 ? bspan : ldb;
    if (!flag) prev = nullptr;
    // few output tiles and a long inner loop: split the inner loop over eight
    // waves (a partial last column chunk goes to the edge tiles)
    constexpr int KCW = 16, KS = 8;
    const int64_t tiles16 = ((R + kRW - 1) / kRW) * (N / KCW);
    if (tiles16 > 0 && tiles16 <= 2048 && K >= 256 && K <= INT32_MAX) {
        const int kq = (int)((K + KS * 32 - 1) / (KS * 32) * 32);
        hipLaunchKernelGGL((k_ad32_mul_ksplit<KCW, KS>),
                           dim3((unsigned)(N / KCW), (unsigned)((R + kRW - 1) / kRW)),
                           dim3(64 * KS), 0, stream, C, ldc, A, lda, B, ldb, R, (int)K, kq,
                           accumulate ? 1 : 0, gate, prev, flag);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess || N % KCW == 0) return e;
        const unsigned gy = (unsigned)((R + 4 * kRW - 1) / (4 * kRW));
        hipLaunchKernelGGL((k_ad32_mul<KCW, false>), dim3(1u, gy), dim3(256), 0, stream, C, ldc,
                           A, lda, B, ldb, R, (int)K, N, N / KCW * KCW, accumulate ? 1 : 0, bmax,
                           gate, prev, flag);
        return hipGetLastError();
    }
    // 16-column tiles when 32-column ones would leave the chip short of waves
    const int64_t waves32 = ((R + kRW - 1) / kRW) * ((N + 31) / 32);
    if (waves32 >= 8192)
        return mul_cw<32>(C, ldc, A, lda, B, ldb, R, K, N, accumulate, bmax, gate, prev, flag,
                          stream);
    return mul_cw<16>(C, ldc, A, lda, B, ldb, R, K, N, accumulate, bmax, gate, prev, flag, stream);
}

hipError_t launch_ad32_mul_group(const MulDesc32 *d, int n, bool acc, hipStream_t st) {
    constexpr int KCW = 16, KS = 8;
    int64_t tiles = 0;
    bool ok = n >= 2 && n <= 4;
    for (int q = 0; q < n && ok; q++) {
        ok = d[q].R > 0 && d[q].K >= 256 && d[q].N >= KCW && d[q].K <= INT32_MAX;
        tiles += ((d[q].R + kRW - 1) / kRW) * (d[q].N / KCW);
    }
    if (!ok || tiles > 2048) {
        for (int q = 0; q < n; q++) {
            if (d[q].R <= 0 || d[q].K <= 0 || d[q].N <= 0) continue;
            hipError_t e = launch_ad32_mul(d[q].C, d[q].ldc, d[q].A, d[q].lda, d[q].B, d[q].ldb,
                                           d[q].R, d[q].K, d[q].N, acc, st, d[q].bspan);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    Ksplit32Group g{};
    g.n = n;
    g.accumulate = acc ? 1 : 0;
    int end = 0;
    for (int q = 0; q < n; q++) {
        Ksplit32Problem &p = g.p[q];
        p.C = d[q].C;
        p.A = d[q].A;
        p.B = d[q].B;
        p.ldc = d[q].ldc;
        p.lda = d[q].lda;
        p.ldb = d[q].ldb;
        p.R = d[q].R;
        p.K = (int)d[q].K;
        p.kq = (int)((d[q].K + KS * 32 - 1) / (KS * 32) * 32);
        p.nx = (int)(d[q].N / KCW);
        end += p.nx * (int)((d[q].R + kRW - 1) / kRW);
        p.end = end;
    }
    hipLaunchKernelGGL((k_ad32_mul_ksplit_group<KCW, KS>), dim3((unsigned)end), dim3(64 * KS), 0,
                       st, g);
    hipError_t e = hipGetLastError();
    // the partial last column chunks, as in launch_ad32_mul
    for (int q = 0; q < n && e == hipSuccess; q++) {
        if (d[q].N % KCW == 0) continue;
        const unsigned gy = (unsigned)((d[q].R + 4 * kRW - 1) / (4 * kRW));
        const int64_t bmax = d[q].bspan >= 0 ? d[q].bspan : d[q].ldb;
        hipLaunchKernelGGL((k_ad32_mul<KCW, false>), dim3(1u, gy), dim3(256), 0, st, d[q].C,
                           d[q].ldc, d[q].A, d[q].lda, d[q].B, d[q].ldb, d[q].R, (int)d[q].K,
                           d[q].N, d[q].N / KCW * KCW, acc ? 1 : 0, bmax, (const int *)nullptr,
                           (const uint32_t *)nullptr, (int *)nullptr);
        e = hipGetLastError();
    }
    return e;
}

hipError_t launch_ad32_closure(uint32_t *T, int64_t ld, int64_t D, bool serial,
                               hipStream_t stream, bool aux_create) {
    static_assert(kPanCW == 2 * dev::kPanelNW, "panel chunking of panel_wgs");
    return closure32(T, ld, D, serial, stream, aux_create);
}

hipError_t launch_ad32_closure_batched_resident(const BatchPlan *plan, int64_t count,
                                                const void *dev_buf, bool dual, bool reflexive,
                                                hipStream_t st) {
    if (count <= 0) return hipSuccess;
    const BatchDesc *desc = static_cast<const BatchDesc *>(dev_buf);
    const BatchItem *items = reinterpret_cast<const BatchItem *>(
        static_cast<const char *>(dev_buf) + batch_desc_bytes(count));
    const unsigned ng = (unsigned)count;
    const dim3 conv(ng, (unsigned)std::max(1, (batch_plan_max_d(plan) + 31) / 32));
    if (dual) hipLaunchKernelGGL(k_batch32_not, conv, dim3(256), 0, st, desc);
    const int xmap = bdev::kXcdChunk;
    hipError_t e;
    for (int kb = 0; kb < batch_plan_rounds(plan); kb++) {
        const BatchLaunch a = batch_plan_phase(plan, 0, kb), b = batch_plan_phase(plan, 1, kb),
                          c = batch_plan_phase(plan, 2, kb);
        if (a.n_wg > 0)
            hipLaunchKernelGGL(k_batch32_pivot, dim3(a.n_wg), dim3(256), 0, st, desc,
                               items + a.offset, kb);
        if (b.n_wg > 0)
            hipLaunchKernelGGL(k_batch32_panels, dim3(b.n_wg), dim3(256), 0, st, desc,
                               items + b.offset, b.n_items + 1, kb, xmap);
        if (c.n_wg > 0)
            hipLaunchKernelGGL(k_batch32_update, dim3(c.n_wg), dim3(256), 0, st, desc,
                               items + c.offset, c.n_items + 1, kb, c.n_units, xmap);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (dual) hipLaunchKernelGGL(k_batch32_not, conv, dim3(256), 0, st, desc);
    // the multiplicative identity's diagonal: S (anti-distance), 0 (distance)
    if (reflexive)
        hipLaunchKernelGGL(k_batch32_diag, dim3(ng), dim3(256), 0, st, desc,
                           dual ? 0u : 0xFFFFFFFFu);
    return hipGetLastError();
}

}  // namespace sr
