// Anti-distance semiring product and blocked Floyd-Warshall closure on
// gfx950 (16-bit storage; uint8 data are widened by the caller into the
// binary16 working form of sr_tiles.h).
//
// Product (Sec. II multiplication algorithm with the Sec. III operations):
//   C (+)= sum over k of (column k of A) times (row k of B).
// Closure (Sec. II Warshall / Sec. III Floyd): the k loop is blocked in
// rounds of kAdBlock pivots.  Round kb with pivot block K:
//   1. pivot:  T_KK := closure of T_KK (one workgroup, registers + LDS);
//   2. panels: T_Kj (+)= T_KK * T_Kj and T_iK (+)= T_iK * T_KK for j, i not in K;
//   3. update: T_ij (+)= T_iK * T_Kj for i, j not in K.
// After round kb every entry is the best path whose intermediate vertices
// lie in blocks 0..kb, exactly the invariant of the unblocked loop after its
// k-th pivot; the result is bit-identical to Warshall's order.  Phases 2 and 3
// are products with accumulation; in phase 2 the output tile is also an
// operand, which is safe because T_KK is closed (T_KK * T_KK <= T_KK): any mix
// of old and new operand entries yields the same result.  The kernels still
// order all reads of a panel tile before its writes with a barrier.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <stdio.h>
#include <stdlib.h>

#include <algorithm>

#include "sr_internal.h"
#include "sr_tiles.h"

namespace sr {
namespace {

using dev::fw_panels_wg;
using dev::fw_update_wg;
using dev::kPanelNW;
using dev::Rect;
using dev::tile_closure;
using dev::u16x2;
using dev::wave_tile;
using dev::wave_tile_body;


// ---------------------------------------------------------------------------
// Product: each wave owns 64*TM rows x 2NW columns; the four waves of a
// workgroup are stacked along the rows and share the column chunk, so they
// read the same B segments through the scalar cache.
// FULL: every column chunk of the grid has all 2NW columns (the launcher
// sends a partial last chunk to a separate FULL = false launch), so the hot
// kernel carries no edge code.  col_base: first column of chunk 0; bmax:
// entries of each B row readable from B (the edge tiles may read a whole
// segment past N, never past bmax).
template <int TM, int NW, bool S8, bool FULL>
__global__ void __launch_bounds__(256)
k_ad_mul(uint16_t *C, int64_t ldc, const uint16_t *A, int64_t lda, const uint16_t *B,
         int64_t ldb, int64_t R, int K, int64_t N, int64_t col_base, int accumulate,
         int64_t bmax, const int *gate, const uint16_t *prev, int *flag) {
    constexpr int CW = 2 * NW, RW = 64 * TM;
    if (gate && *gate == 0) return;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform per wave
    const int64_t row0 = ((int64_t)blockIdx.y * 4 + wave) * RW;
    const int64_t col0 = col_base + (int64_t)blockIdx.x * CW;
    if (row0 >= R) return;
    const int nrows = (int)min<int64_t>(RW, R - row0);
    const int ncols = FULL ? CW : (int)min<int64_t>(CW, N - col0);
    if (FULL) {
        wave_tile_body<TM, NW, S8, true>(C + row0 * ldc + col0, ldc, A + row0 * lda, lda,
                                         B + col0, ldb, nrows, CW, K, accumulate != 0, false);
    } else {
        wave_tile<TM, NW, S8>(C + row0 * ldc + col0, ldc, A + row0 * lda, lda, B + col0, ldb,
                              nrows, ncols, bmax - col0, K, accumulate != 0, false);
    }
    if (prev) {
        // change check: this lane's rows of the tile just stored, read back,
        // against the same entries of prev (same layout as C)
        const int lane = threadIdx.x & 63;
        bool diff = false;
        for (int t = 0; t < TM; t++) {
            const int r = lane + 64 * t;
            if (r >= nrows) break;
            const uint16_t *c = C + (row0 + r) * ldc + col0;
            const uint16_t *p = prev + (row0 + r) * ldc + col0;
            for (int j = 0; j < ncols; j++) diff |= c[j] != p[j];
        }
        if (__any(diff) && lane == 0) *flag = 1;
    }
}

// Product with the inner dimension split over the KS waves of a workgroup,
// for products with too few output tiles to fill the chip: all KS waves take
// the same 64-row x 2NW-column tile of C (every chunk of the launch has all
// 2NW columns inside N), wave w the inner steps [w kq, (w + 1) kq) (kq a
// multiple of 32); their partial results meet in LDS, where the (+) of the
// KS partials (and of C when accumulating) is taken.  (+) is max, so
// splitting the inner loop changes nothing in the result.  All partials are
// >= 0, so the max of their 16-bit patterns is their max also in the
// binary16 form.
template <int NW, int KS, bool S8>
__device__ __forceinline__ void ksplit_tile(uint4 (*part)[64][NW / 4], uint16_t *C, int64_t ldc,
                                            const uint16_t *A, int64_t lda, const uint16_t *B,
                                            int64_t ldb, int64_t R, int K, int kq, int accumulate,
                                            const uint16_t *prev, int *flag, int64_t row0,
                                            int64_t col0) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform per wave
    const int nrows = (int)min<int64_t>(64, R - row0);
    const int k0 = min(K, wave * kq), k1 = min(K, k0 + kq);
    // this wave's partial product (rows >= nrows are not written)
    wave_tile_body<1, NW, S8, true>(reinterpret_cast<uint16_t *>(&part[wave][0][0]), 2 * NW,
                                    A + row0 * lda + k0, lda, B + (int64_t)k0 * ldb + col0, ldb,
                                    nrows, 2 * NW, k1 - k0, false, false);
    __syncthreads();
    // (+) of the partials, one 32-bit word (two entries) per thread and pass;
    // with prev, each word is also compared with the same word of prev
    bool diff = false;
    for (int wi = threadIdx.x; wi < 64 * NW; wi += 64 * KS) {
        const int row = wi / NW, word = wi % NW;
        if (row >= nrows) continue;
        u16x2 v = dev::as_pair(reinterpret_cast<const uint32_t *>(&part[0][row][0])[word]);
#pragma unroll
        for (int q = 1; q < KS; q++)
            v = __builtin_elementwise_max(
                v, dev::as_pair(reinterpret_cast<const uint32_t *>(&part[q][row][0])[word]));
        uint32_t *dst = reinterpret_cast<uint32_t *>(C + (row0 + row) * ldc + col0) + word;
        if (accumulate) v = __builtin_elementwise_max(v, dev::as_pair(*dst));
        *dst = dev::as_word(v);
        if (prev)
            diff |= dev::as_word(v) !=
                    reinterpret_cast<const uint32_t *>(prev + (row0 + row) * ldc + col0)[word];
    }
    if (prev && __any(diff) && (threadIdx.x & 63) == 0) *flag = 1;
}

template <int NW, int KS, bool S8>
__global__ void __launch_bounds__(64 * KS)
k_ad_mul_ksplit(uint16_t *C, int64_t ldc, const uint16_t *A, int64_t lda, const uint16_t *B,
                int64_t ldb, int64_t R, int K, int kq, int accumulate, const int *gate,
                const uint16_t *prev, int *flag) {
    __shared__ uint4 part[KS][64][NW / 4];
    if (gate && *gate == 0) return;  // (uniform over the workgroup: before any barrier)
    ksplit_tile<NW, KS, S8>(part, C, ldc, A, lda, B, ldb, R, K, kq, accumulate, prev, flag,
                            (int64_t)blockIdx.y * 64, (int64_t)blockIdx.x * 2 * NW);
}

// Up to four independent products C_q (+)= A_q * B_q in one launch of the
// K-split tiles above (the panels, or the blocks of a big-block round, which
// are each too small to fill the chip): workgroups [end_{q-1}, end_q) take
// the nx_q x ny_q tiles of product q, row-major.  No product's output may be
// another's operand; a product's output may be its own operand where the
// single-product kernel allows it.
struct KsplitProblem {
    uint16_t *C;
    const uint16_t *A, *B;
    int64_t ldc, lda, ldb, R;
    int K, kq, nx, end;
};
struct KsplitGroup {
    KsplitProblem p[4];
    int n, accumulate;
};

template <int NW, int KS, bool S8>
__global__ void __launch_bounds__(64 * KS) k_ad_mul_ksplit_group(KsplitGroup g) {
    __shared__ uint4 part[KS][64][NW / 4];
    const int b = blockIdx.x;
    int q = 0;
    while (q + 1 < g.n && b >= g.p[q].end) q++;
    const KsplitProblem &p = g.p[q];
    const int local = b - (q > 0 ? g.p[q - 1].end : 0);
    ksplit_tile<NW, KS, S8>(part, p.C, p.ldc, p.A, p.lda, p.B, p.ldb, p.R, p.K, p.kq,
                            g.accumulate, nullptr, nullptr, (int64_t)(local / p.nx) * 64,
                            (int64_t)(local % p.nx) * 2 * NW);
}

template <bool S8>
__global__ void __launch_bounds__(256)
k_ad_fw_pivot(uint16_t *T, int64_t ld, int64_t k0, int bs, int prio) {
    if (prio) __builtin_amdgcn_s_setprio(2);
    __shared__ uint32_t lds_row[2 * 128];
    __shared__ uint32_t lds_col[2 * 128];
    tile_closure<S8>(T + k0 * ld + k0, ld, bs, lds_row, lds_col);
}

// Phase 2 (the workgroup body is fw_panels_wg in sr_tiles.h).
template <bool S8>
__global__ void __launch_bounds__(256)
k_ad_fw_panels(uint16_t *T, int64_t ld, int D, int k0, int bs, int n_rowwg, int prio) {
    if (prio) __builtin_amdgcn_s_setprio(2);
    fw_panels_wg<S8>(T, ld, D, k0, bs, n_rowwg, (int)blockIdx.x);
}

// Phase 3 over a rectangle of tiles (body: fw_update_wg in sr_tiles.h).
// FULL: every selected column chunk has all 2NW columns inside D (the
// launcher sends a partial last chunk to a FULL = false launch).
template <int TM, int NW, bool S8, bool FULL>
__global__ void __launch_bounds__(256)
k_ad_fw_update(uint16_t *T, int64_t ld, int D, int k0, int bs, Rect q, int prio) {
    if (prio) __builtin_amdgcn_s_setprio(2);
    fw_update_wg<TM, NW, S8, FULL>(T, ld, D, k0, bs, q, (int)blockIdx.x, (int)blockIdx.y);
}

// The lookahead part A(kb) of a round (the update of row block kb+1 and of
// column block kb+1, which the next round's pivot and panels wait for) in one
// launch of short waves: tiles of 64 rows x 32 columns, workgroups [0, nta)
// taking the tiles of rectangle qa and the rest those of qb (Rect semantics
// of fw_update_wave, one tile per workgroup, column-chunk major).  The four
// waves of a workgroup split the bs inner steps of their tile; their partial
// results meet in LDS, where the (+) of the four and of the tile is stored.
// (The same tiles as whole-K waves ran at one wave per SIMD, latency-bound.)
// The tiles it writes are never its operands (those lie in row and column
// block kb).  A partial last column chunk runs as one whole-K wave.
template <bool S8>
__global__ void __launch_bounds__(256)
k_ad_fw_lookahead(uint16_t *T, int64_t ld, int D, int k0, int bs, Rect qa, int nta, Rect qb,
                  int prio) {
    if (prio) __builtin_amdgcn_s_setprio(2);
    constexpr int NW = 16;  // packed pairs per row of a tile (32 columns)
    __shared__ uint4 part[4][64][NW / 4];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int t = (int)blockIdx.x;
    const bool in_a = t < nta;
    const Rect q = in_a ? qa : qb;
    if (!in_a) t -= nta;
    const int nr = (q.r_hi - q.r_lo) - (q.r_ex1 - q.r_ex0);
    int rc = q.r_lo + t % nr;
    if (rc >= q.r_ex0) rc += q.r_ex1 - q.r_ex0;
    int c = q.c_lo + t / nr;
    if (c >= q.c_ex0) c += q.c_ex1 - q.c_ex0;
    if (rc >= q.r_hi || c >= q.c_hi) return;  // (the grid has no such tile)
    const int64_t row0 = (int64_t)rc * 64, col0 = (int64_t)c * 2 * NW;
    const int nrows = (int)min<int64_t>(64, (int64_t)D - row0);
    const int ncols = (int)min<int64_t>(2 * NW, (int64_t)D - col0);
    uint16_t *C = T + row0 * ld + col0;
    const uint16_t *A = T + row0 * ld + k0;
    const uint16_t *B = T + (int64_t)k0 * ld + col0;
    if (ncols < 2 * NW) {
        if (wave == 0)
            wave_tile<1, NW, S8>(C, ld, A, ld, B, ld, nrows, ncols, ld - col0, bs, true, false);
        return;
    }
    const int kq = (bs + 4 * 8 - 1) / (4 * 8) * 8;  // a multiple of 8 entries (16 bytes)
    const int kk0 = min(bs, wave * kq), kk1 = min(bs, kk0 + kq);
    wave_tile_body<1, NW, S8, true>(reinterpret_cast<uint16_t *>(&part[wave][0][0]), 2 * NW,
                                    A + kk0, ld, B + (int64_t)kk0 * ld, ld, nrows, 2 * NW,
                                    kk1 - kk0, false, false);
    __syncthreads();
    for (int wi = threadIdx.x; wi < 64 * NW; wi += 256) {
        const int row = wi / NW, word = wi % NW;
        if (row >= nrows) continue;
        u16x2 v = dev::as_pair(reinterpret_cast<const uint32_t *>(&part[0][row][0])[word]);
#pragma unroll
        for (int w = 1; w < 4; w++)
            v = __builtin_elementwise_max(
                v, dev::as_pair(reinterpret_cast<const uint32_t *>(&part[w][row][0])[word]));
        uint32_t *dst = reinterpret_cast<uint32_t *>(C + (int64_t)row * ld) + word;
        *dst = dev::as_word(__builtin_elementwise_max(v, dev::as_pair(*dst)));
    }
}

// uint8 <-> the 16-bit working form of uint8 data (binary16 values, see
// sr_tiles.h), 8 entries per thread; rows padded with zeros up to the next
// multiple of 8 in the destination of a widening.
__global__ void __launch_bounds__(256)
k_widen(uint16_t *dst, int64_t ldd, const uint8_t *src, int64_t lds, int64_t R, int64_t C) {
    const int64_t gpr = (C + 7) >> 3;
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= R * gpr) return;
    const int64_t row = g / gpr, c0 = (g % gpr) * 8;
    const uint8_t *s = src + row * lds + c0;
    uint16_t v[8];
    if (c0 + 8 <= C) {
        const uint2 w = *reinterpret_cast<const uint2 *>(s);
#pragma unroll
        for (int i = 0; i < 4; i++) {
            v[i] = dev::u8_to_work((w.x >> (8 * i)) & 0xFFu);
            v[4 + i] = dev::u8_to_work((w.y >> (8 * i)) & 0xFFu);
        }
    } else {
#pragma unroll
        for (int i = 0; i < 8; i++) v[i] = (c0 + i < C) ? dev::u8_to_work(s[i]) : (uint16_t)0;
    }
    uint4 o;
    o.x = v[0] | ((uint32_t)v[1] << 16);
    o.y = v[2] | ((uint32_t)v[3] << 16);
    o.z = v[4] | ((uint32_t)v[5] << 16);
    o.w = v[6] | ((uint32_t)v[7] << 16);
    *reinterpret_cast<uint4 *>(dst + row * ldd + c0) = o;
}

__global__ void __launch_bounds__(256)
k_narrow(uint8_t *dst, int64_t ldd, const uint16_t *src, int64_t lds, int64_t R, int64_t C) {
    const int64_t gpr = (C + 7) >> 3;
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= R * gpr) return;
    const int64_t row = g / gpr, c0 = (g % gpr) * 8;
    const uint4 w = *reinterpret_cast<const uint4 *>(src + row * lds + c0);
    const uint32_t ww[4] = {w.x, w.y, w.z, w.w};
    uint8_t b[8];
#pragma unroll
    for (int i = 0; i < 8; i++) b[i] = dev::work_to_u8((uint16_t)(ww[i >> 1] >> (16 * (i & 1))));
    uint8_t *d = dst + row * ldd + c0;
    if (c0 + 8 <= C) {
        uint2 o;
        o.x = b[0] | ((uint32_t)b[1] << 8) | ((uint32_t)b[2] << 16) | ((uint32_t)b[3] << 24);
        o.y = b[4] | ((uint32_t)b[5] << 8) | ((uint32_t)b[6] << 16) | ((uint32_t)b[7] << 24);
        *reinterpret_cast<uint2 *>(d) = o;
    } else {
        for (int i = 0; i < 8; i++)
            if (c0 + i < C) d[i] = b[i];
    }
}

// Tile shape of the product: rows per lane and column pairs per wave.  Wider
// tiles amortise the per-step work that is not a packed update and reuse each
// scalar-loaded B word for more updates; narrower ones give more waves for
// small products.
struct Shape {
    int tm, nw;
};
template <int TM, int NW>
struct ShapeT {
    static constexpr int tm = TM, nw = NW;
};

Shape pick_mul_shape(int64_t R, int64_t N) {
    const Shape cand[] = {{2, 32}, {1, 32}, {1, 16}, {1, 8}};
    for (const Shape &s : cand) {
        const int64_t waves = ((R + 64 * s.tm - 1) / (64 * s.tm)) * ((N + 2 * s.nw - 1) / (2 * s.nw));
        if (waves >= 8192) return s;
    }
    return Shape{1, 8};
}

template <int TM, int NW, bool S8>
hipError_t mul_shape(uint16_t *C, int64_t ldc, const uint16_t *A, int64_t lda, const uint16_t *B,
                     int64_t ldb, int64_t R, int64_t K, int64_t N, bool acc, int64_t bmax,
                     const int *gate, const uint16_t *prev, int *flag, hipStream_t st) {
    constexpr int CW = 2 * NW;
    const unsigned gy = (unsigned)((R + 256 * TM - 1) / (256 * TM));
    const int64_t nfull = N / CW;
    if (nfull > 0) {
        hipLaunchKernelGGL((k_ad_mul<TM, NW, S8, true>), dim3((unsigned)nfull, gy), dim3(256), 0,
                           st, C, ldc, A, lda, B, ldb, R, (int)K, N, (int64_t)0, acc ? 1 : 0,
                           bmax, gate, prev, flag);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (N % CW) {
        // the partial last chunk, as 16-column tiles of one row per lane
        const int64_t c0 = nfull * CW;
        const unsigned gx = (unsigned)((N - c0 + 15) / 16);
        hipLaunchKernelGGL((k_ad_mul<1, 8, S8, false>), dim3(gx, (unsigned)((R + 255) / 256)),
                           dim3(256), 0, st, C, ldc, A, lda, B, ldb, R, (int)K, N, c0,
                           acc ? 1 : 0, bmax, gate, prev, flag);
        return hipGetLastError();
    }
    return hipSuccess;
}

// Products with at most 2048 output tiles of 64 x 16 (two waves per SIMD or
// fewer) but a long inner dimension: 16-column tiles with the inner loop split
// over the KS waves of a workgroup (k_ad_mul_ksplit); a partial last column
// chunk goes to the edge kernel.  These launches are latency-bound: with at
// most 256 tiles (one workgroup per compute unit) sixteen waves split the
// inner loop, which halves each wave's chain of scalar-load waits; with more
// tiles eight (measured on 512 x 512 x 512 products and the big-block
// closure of a sparse 1024-vertex graph: 175 against 184 us; 1024^3: 39
// against 46 us).
template <bool S8, int KS>
hipError_t mul_ksplit_ks(uint16_t *C, int64_t ldc, const uint16_t *A, int64_t lda,
                         const uint16_t *B, int64_t ldb, int64_t R, int64_t K, int64_t N,
                         bool acc, int64_t bmax, const int *gate, const uint16_t *prev, int *flag,
                         hipStream_t st) {
    constexpr int NW = 8, CW = 2 * NW;
    const int64_t nfull = N / CW;
    const int kq = (int)((K + KS * 32 - 1) / (KS * 32) * 32);
    if (nfull > 0) {
        hipLaunchKernelGGL((k_ad_mul_ksplit<NW, KS, S8>),
                           dim3((unsigned)nfull, (unsigned)((R + 63) / 64)), dim3(64 * KS), 0, st,
                           C, ldc, A, lda, B, ldb, R, (int)K, kq, acc ? 1 : 0, gate, prev,
                           flag);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (N % CW) {
        const int64_t c0 = nfull * CW;
        hipLaunchKernelGGL((k_ad_mul<1, 8, S8, false>), dim3(1u, (unsigned)((R + 255) / 256)),
                           dim3(256), 0, st, C, ldc, A, lda, B, ldb, R, (int)K, N, c0,
                           acc ? 1 : 0, bmax, gate, prev, flag);
        return hipGetLastError();
    }
    return hipSuccess;
}

template <bool S8>
hipError_t mul_ksplit(uint16_t *C, int64_t ldc, const uint16_t *A, int64_t lda,
                      const uint16_t *B, int64_t ldb, int64_t R, int64_t K, int64_t N, bool acc,
                      int64_t bmax, const int *gate, const uint16_t *prev, int *flag,
                      hipStream_t st) {
    const int64_t tiles = ((R + 63) / 64) * (N / 16);
    if (tiles <= 256)
        return mul_ksplit_ks<S8, 16>(C, ldc, A, lda, B, ldb, R, K, N, acc, bmax, gate, prev, flag,
                                     st);
    return mul_ksplit_ks<S8, 8>(C, ldc, A, lda, B, ldb, R, K, N, acc, bmax, gate, prev, flag, st);
}

template <bool S8>
hipError_t mul_s(uint16_t *C, int64_t ldc, const uint16_t *A, int64_t lda, const uint16_t *B,
                 int64_t ldb, int64_t R, int64_t K, int64_t N, bool acc, int64_t bmax,
                 const int *gate, const uint16_t *prev, int *flag, hipStream_t st) {
    const int64_t tiles16 = ((R + 63) / 64) * (N / 16);
    if (tiles16 > 0 && tiles16 <= 2048 && K >= 256)
        return mul_ksplit<S8>(C, ldc, A, lda, B, ldb, R, K, N, acc, bmax, gate, prev, flag, st);
    const Shape s = pick_mul_shape(R, N);
    auto run = [&](auto shape) {
        constexpr int TM = decltype(shape)::tm, NW = decltype(shape)::nw;
        return mul_shape<TM, NW, S8>(C, ldc, A, lda, B, ldb, R, K, N, acc, bmax, gate, prev, flag,
                                     st);
    };
    if (s.tm == 2) return run(ShapeT<2, 32>{});
    switch (s.nw) {
        case 32: return run(ShapeT<1, 32>{});
        case 16: return run(ShapeT<1, 16>{});
        default: return run(ShapeT<1, 8>{});
    }
}

// Several products in one K-split launch when each has a long enough inner
// dimension and together they have at most 2048 output tiles of 64 x 16
// (the K-split rule of mul_s); otherwise one launch each.
template <bool S8>
hipError_t mul_group_s(const MulDesc *d, int n, bool acc, hipStream_t st) {
    constexpr int NW = 8, CW = 2 * NW, KS = 8;
    int64_t tiles = 0;
    bool ok = n >= 2 && n <= 4;
    for (int q = 0; q < n && ok; q++) {
        ok = d[q].R > 0 && d[q].K >= 256 && d[q].N >= CW && d[q].K <= INT32_MAX;
        tiles += ((d[q].R + 63) / 64) * (d[q].N / CW);
    }
    if (!ok || tiles > 2048) {
        for (int q = 0; q < n; q++) {
            if (d[q].R <= 0 || d[q].K <= 0 || d[q].N <= 0) continue;
            hipError_t e = mul_s<S8>(d[q].C, d[q].ldc, d[q].A, d[q].lda, d[q].B, d[q].ldb, d[q].R,
                                     d[q].K, d[q].N, acc, d[q].bspan >= 0 ? d[q].bspan : d[q].ldb,
                                     nullptr, nullptr, nullptr, st);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    KsplitGroup g{};
    g.n = n;
    g.accumulate = acc ? 1 : 0;
    int end = 0;
    for (int q = 0; q < n; q++) {
        KsplitProblem &p = g.p[q];
        p.C = d[q].C;
        p.A = d[q].A;
        p.B = d[q].B;
        p.ldc = d[q].ldc;
        p.lda = d[q].lda;
        p.ldb = d[q].ldb;
        p.R = d[q].R;
        p.K = (int)d[q].K;
        p.kq = (int)((d[q].K + KS * 32 - 1) / (KS * 32) * 32);
        p.nx = (int)(d[q].N / CW);
        end += p.nx * (int)((d[q].R + 63) / 64);
        p.end = end;
    }
    hipLaunchKernelGGL((k_ad_mul_ksplit_group<NW, KS, S8>), dim3((unsigned)end), dim3(64 * KS), 0,
                       st, g);
    hipError_t e = hipGetLastError();
    // the partial last column chunks, as in mul_ksplit
    for (int q = 0; q < n && e == hipSuccess; q++) {
        if (d[q].N % CW == 0) continue;
        const int64_t c0 = d[q].N / CW * CW;
        hipLaunchKernelGGL((k_ad_mul<1, 8, S8, false>), dim3(1u, (unsigned)((d[q].R + 255) / 256)),
                           dim3(256), 0, st, d[q].C, d[q].ldc, d[q].A, d[q].lda, d[q].B, d[q].ldb,
                           d[q].R, (int)d[q].K, d[q].N, c0, acc ? 1 : 0,
                           d[q].bspan >= 0 ? d[q].bspan : d[q].ldb, (const int *)nullptr,
                           (const uint16_t *)nullptr, (int *)nullptr);
        e = hipGetLastError();
    }
    return e;
}

// ---------------------------------------------------------------------------
// Closure driver.
//
// Per round kb: pivot(kb), panels(kb), then the update of every tile outside
// row block kb and column block kb.  With lookahead the update is split:
//   A(kb): the tiles of row block kb+1 and column block kb+1 (outside block
//          kb), i.e. next round's pivot and panels;
//   B(kb): the rest (outside blocks kb and kb+1).
// pivot(kb+1) and panels(kb+1) need only A(kb), so they run on the caller's
// stream while B(kb) runs on a second stream; they touch disjoint tiles (and
// B(kb) reads no tile that panels(kb+1) writes).  A(kb+1) waits for B(kb).
// The critical path per round is A + pivot + panels; the bulk of the work
// (B) overlaps it.
// ---------------------------------------------------------------------------
struct Plan {
    int64_t D;
    int tm, nw;
    int rw, cw;      // rows / columns of a row / column chunk
    int nrc, ncc;    // number of row / column chunks
};

// Update-tile shapes compiled in (rows per lane, column pairs per wave); a
// row chunk (64 * rows per lane) must not exceed the pivot block.
bool tile_supported(int tm, int nw) {
    return (tm == 1 || tm == 2) && (nw == 8 || nw == 16 || nw == 32);
}

// Tuning overrides, read once: SR_AD_TILE="tm,nw" forces the update tile
// shape (2,32 | 1,32 | 1,16 | 1,8); SR_LOOKAHEAD=0 disables the second stream.
struct Overrides {
    int tm = 0, nw = 0;
    bool lookahead = true;
    bool prio = true;  // raise the wave priority of the critical-path kernels
    bool split_lookahead = true;  // A(kb) as one launch of K-split tiles
    Overrides() {
        if (const char *t = getenv("SR_AD_TILE")) {
            int a = 0, b = 0;
            if (sscanf(t, "%d,%d", &a, &b) == 2 && tile_supported(a, b)) {
                tm = a;
                nw = b;
            }
        }
        if (const char *l = getenv("SR_LOOKAHEAD")) lookahead = atoi(l) != 0;
        if (const char *v = getenv("SR_PRIO")) prio = atoi(v) != 0;
        if (const char *v = getenv("SR_SPLIT_LOOKAHEAD")) split_lookahead = atoi(v) != 0;
    }
};

const Overrides &overrides() {
    static const Overrides o;
    return o;
}

Plan make_plan(int64_t D) {
    Plan p;
    p.D = D;
    if (D >= 2048) {
        p.tm = 1;
        p.nw = 16;
    } else if (D >= 512) {
        p.tm = 1;
        p.nw = 16;
    } else {
        p.tm = 1;
        p.nw = 8;
    }
    if (overrides().tm) {
        p.tm = overrides().tm;
        p.nw = overrides().nw;
    }
    p.rw = 64 * p.tm;
    p.cw = 2 * p.nw;
    p.nrc = (int)((D + p.rw - 1) / p.rw);
    p.ncc = (int)((D + p.cw - 1) / p.cw);
    return p;
}

int blocks_of(int64_t D) { return (int)((D + kAdBlock - 1) / kAdBlock); }
int block_k0(int64_t kb) { return (int)(kb * kAdBlock); }
int block_bs(int64_t D, int64_t kb) { return (int)std::min<int64_t>(kAdBlock, D - kb * kAdBlock); }

// chunks [lo, hi) covering block kb at chunk width w
void block_chunks(int64_t D, int64_t kb, int w, int *lo, int *hi) {
    const int k0 = block_k0(kb), bs = block_bs(D, kb);
    *lo = k0 / w;
    *hi = (k0 + bs + w - 1) / w;
}

template <int TM, int NW, bool S8, bool FULL>
hipError_t update_launch(uint16_t *T, int64_t ld, int64_t D, int k0, int bs, const Rect &q,
                         int prio, hipStream_t st) {
    const int nr = (q.r_hi - q.r_lo) - (q.r_ex1 - q.r_ex0);
    const int nc = (q.c_hi - q.c_lo) - (q.c_ex1 - q.c_ex0);
    if (nr <= 0 || nc <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_ad_fw_update<TM, NW, S8, FULL>), dim3(nc, (nr + 3) / 4), dim3(256), 0,
                       st, T, ld, (int)D, k0, bs, q, prio);
    return hipGetLastError();
}

// The rectangle's full column chunks go to the hot kernel; a partial last
// chunk of the matrix (D not a multiple of 2NW), if selected, goes to the
// edge kernel as 16-column tiles of 64 rows.
template <int TM, int NW, bool S8>
hipError_t update_rect_t(uint16_t *T, int64_t ld, int64_t D, int k0, int bs, Rect q, int prio,
                         hipStream_t st) {
    constexpr int CW = 2 * NW;
    const int last = (int)((D + CW - 1) / CW) - 1;
    const bool has_partial = (D % CW) != 0 && q.c_lo <= last && last < q.c_hi &&
                             !(q.c_ex0 <= last && last < q.c_ex1);
    if (has_partial) {
        // the last chunk is the final one of the range: drop it from the hot launch
        q.c_hi = last;
        q.c_ex0 = std::min(q.c_ex0, q.c_hi);
        q.c_ex1 = std::min(q.c_ex1, q.c_hi);
    }
    hipError_t e = update_launch<TM, NW, S8, true>(T, ld, D, k0, bs, q, prio, st);
    if (e != hipSuccess || !has_partial) return e;
    Rect edge;
    const int r64 = (int)((D + 63) / 64);
    edge.r_lo = std::min(q.r_lo * TM, r64);
    edge.r_hi = std::min(q.r_hi * TM, r64);
    edge.r_ex0 = std::min(q.r_ex0 * TM, edge.r_hi);
    edge.r_ex1 = std::min(q.r_ex1 * TM, edge.r_hi);
    edge.c_lo = last * CW / 16;
    edge.c_hi = (int)((D + 15) / 16);
    edge.c_ex0 = edge.c_ex1 = edge.c_hi;
    return update_launch<1, 8, S8, false>(T, ld, D, k0, bs, edge, prio, st);
}

template <bool S8>
hipError_t update_rect(const Plan &p, uint16_t *T, int64_t ld, int64_t kb, Rect q,
                       hipStream_t st, double units, bool critical = false) {
    const int prio = critical && overrides().prio ? 1 : 0;
    // an empty exclusion is placed at the end of the range
    if (q.r_ex1 <= q.r_ex0) q.r_ex0 = q.r_ex1 = q.r_hi;
    if (q.c_ex1 <= q.c_ex0) q.c_ex0 = q.c_ex1 = q.c_hi;
    const int k0 = block_k0(kb), bs = block_bs(p.D, kb);
    const bool prof = prof_on();
    if (prof) prof_begin(st);
    hipError_t e;
    switch (p.tm * 100 + p.nw) {
        case 232: e = update_rect_t<2, 32, S8>(T, ld, p.D, k0, bs, q, prio, st); break;
        case 216: e = update_rect_t<2, 16, S8>(T, ld, p.D, k0, bs, q, prio, st); break;
        case 208: e = update_rect_t<2, 8, S8>(T, ld, p.D, k0, bs, q, prio, st); break;
        case 132: e = update_rect_t<1, 32, S8>(T, ld, p.D, k0, bs, q, prio, st); break;
        case 116: e = update_rect_t<1, 16, S8>(T, ld, p.D, k0, bs, q, prio, st); break;
        default: e = update_rect_t<1, 8, S8>(T, ld, p.D, k0, bs, q, prio, st); break;
    }
    if (prof) prof_end(st, 1, 2, units);
    return e;
}

// A(kb) as one launch of k_ad_fw_lookahead (plan tiles of 64 x 32).
template <bool S8>
hipError_t lookahead_s(const Plan &p, uint16_t *T, int64_t ld, int64_t kb, Rect qa, Rect qb,
                       double units, hipStream_t st, bool record = true) {
    auto tiles = [](Rect &q) {
        if (q.r_ex1 <= q.r_ex0) q.r_ex0 = q.r_ex1 = q.r_hi;
        if (q.c_ex1 <= q.c_ex0) q.c_ex0 = q.c_ex1 = q.c_hi;
        const int nr = (q.r_hi - q.r_lo) - (q.r_ex1 - q.r_ex0);
        const int nc = (q.c_hi - q.c_lo) - (q.c_ex1 - q.c_ex0);
        return nr > 0 && nc > 0 ? nr * nc : 0;
    };
    const int nta = tiles(qa), ntb = tiles(qb);
    if (nta + ntb == 0) return hipSuccess;
    if (nta == 0) qa = qb;  // (a rectangle with no tiles is never selected)
    const int k0 = block_k0(kb), bs = block_bs(p.D, kb);
    const bool prof = record && prof_on();
    if (prof) prof_begin(st);
    hipLaunchKernelGGL((k_ad_fw_lookahead<S8>), dim3((unsigned)(nta + ntb)), dim3(256), 0, st, T,
                       ld, (int)p.D, k0, bs, qa, nta, qb, overrides().prio ? 1 : 0);
    hipError_t e = hipGetLastError();
    if (prof) prof_end(st, 1, 2, units);
    return e;
}

// Phase 2 as one launch of k_ad_fw_lookahead: the row panel's tiles (rows of
// block kb, columns outside it) and the column panel's (rows outside block
// kb, its columns), four waves splitting the inner steps of each tile.  A
// panel tile is also an operand of its own and of the other panel tiles; that
// is exact because T_KK is closed (any mix of old and new entries gives the
// same result), as in the one-wave-per-tile panel kernel.
template <bool S8>
hipError_t panels_split_s(const Plan &p, uint16_t *T, int64_t ld, int64_t kb, hipStream_t st) {
    int rl, rh, cl, ch;
    block_chunks(p.D, kb, p.rw, &rl, &rh);
    block_chunks(p.D, kb, p.cw, &cl, &ch);
    const double bs = block_bs(p.D, kb);
    const Rect row_panel{rl, rh, rh, rh, 0, p.ncc, cl, ch};
    const Rect col_panel{0, p.nrc, rl, rh, cl, ch, ch, ch};
    const bool prof = prof_on();
    if (prof) prof_begin(st);
    hipError_t e = lookahead_s<S8>(p, T, ld, kb, row_panel, col_panel, 0.0, st, false);
    if (prof) prof_end(st, 1, 1, 2.0 * ((double)p.D - bs) * bs * bs);
    return e;
}

// Whether phase 2 and the lookahead part run as K-split tiles: where the
// chain of pivot, panels and lookahead part is the critical path (the bulk
// update of a round being short), with the plan's 64 x 32 tiles.
bool split_chain(const Plan &p) {
    return p.tm == 1 && p.nw == 16 && overrides().split_lookahead && p.D <= 6144;
}

template <bool S8>
hipError_t pivot_s(uint16_t *T, int64_t ld, int64_t D, int64_t kb, hipStream_t st) {
    const int k0 = block_k0(kb), bs = block_bs(D, kb);
    const bool prof = prof_on();
    if (prof) prof_begin(st);
    hipLaunchKernelGGL((k_ad_fw_pivot<S8>), dim3(1), dim3(256), 0, st, T, ld, (int64_t)k0, bs,
                       overrides().prio ? 1 : 0);
    hipError_t e = hipGetLastError();
    if (prof) prof_end(st, 1, 0, (double)bs * bs * bs);
    return e;
}

template <bool S8>
hipError_t panels_s(uint16_t *T, int64_t ld, int64_t D, int64_t kb, hipStream_t st) {
    const int k0 = block_k0(kb), bs = block_bs(D, kb);
    int n_rowwg = 0, n_colwg = 0;
    dev::panel_wgs(D, k0, bs, &n_rowwg, &n_colwg);
    const int n = n_rowwg + n_colwg;
    if (n <= 0) return hipSuccess;
    const bool prof = prof_on();
    if (prof) prof_begin(st);
    hipLaunchKernelGGL((k_ad_fw_panels<S8>), dim3(n), dim3(256), 0, st, T, ld, (int)D, k0, bs,
                       n_rowwg, overrides().prio ? 1 : 0);
    hipError_t e = hipGetLastError();
    if (prof) prof_end(st, 1, 1, 2.0 * (double)(D - bs) * bs * bs);
    return e;
}

template <bool S8>
hipError_t closure_s(uint16_t *T, int64_t ld, int64_t D, bool serial, hipStream_t st,
                     bool aux_create) {
    const Plan p = make_plan(D);
    const int nb = blocks_of(D);
    hipError_t e = pivot_s<S8>(T, ld, D, 0, st);
    if (e != hipSuccess || nb == 1) return e;
    const bool split = split_chain(p);
    if ((e = split ? panels_split_s<S8>(p, T, ld, 0, st) : panels_s<S8>(T, ld, D, 0, st)) !=
        hipSuccess)
        return e;

    // With a second stream, B(kb) -- the update outside row and column
    // blocks kb+1 -- runs there, queued behind B(kb-1) as soon as panels(kb)
    // is done, and the caller's stream waits for B(kb-1) only before A(kb),
    // the rest of round kb's update.  So B(kb) follows B(kb-1) back to back
    // while the chain A(kb) -> pivot(kb+1) -> panels(kb+1) runs beside it.
    Aux *aux = (nb > 2 && !serial && overrides().lookahead) ? aux_acquire(st, aux_create) : nullptr;
    for (int kb = 0; kb < nb; kb++) {
        int rl, rh, cl, ch;
        block_chunks(D, kb, p.rw, &rl, &rh);
        block_chunks(D, kb, p.cw, &cl, &ch);
        const double bs = block_bs(D, kb);
        if (kb + 1 == nb || !aux) {
            // whole update of round kb (after B(kb-1)), then the next pivot and panels
            if (aux && kb > 0) e = hipStreamWaitEvent(st, aux->ev_aux[(kb - 1) & 1], 0);
            const double rest = (double)D - bs;
            if (e == hipSuccess)
                e = update_rect<S8>(p, T, ld, kb, Rect{0, p.nrc, rl, rh, 0, p.ncc, cl, ch}, st,
                                    rest * rest * bs);
            if (e == hipSuccess && kb + 1 < nb) e = pivot_s<S8>(T, ld, D, kb + 1, st);
            if (e == hipSuccess && kb + 1 < nb)
                e = split ? panels_split_s<S8>(p, T, ld, kb + 1, st)
                          : panels_s<S8>(T, ld, D, kb + 1, st);
            if (e != hipSuccess) break;
            continue;
        }
        int rl1, rh1, cl1, ch1;
        block_chunks(D, kb + 1, p.rw, &rl1, &rh1);
        block_chunks(D, kb + 1, p.cw, &cl1, &ch1);
        const double bs1 = block_bs(D, kb + 1);
        const double rest2 = (double)D - bs - bs1;
        // B(kb) on the second stream, after panels(kb) (recorded on st)
        e = hipEventRecord(aux->ev_main, st);
        if (e == hipSuccess) e = hipStreamWaitEvent(aux->stream, aux->ev_main, 0);
        if (e == hipSuccess)
            e = update_rect<S8>(p, T, ld, kb, Rect{0, p.nrc, rl, rh1, 0, p.ncc, cl, ch1},
                                aux->stream, rest2 * rest2 * bs);
        if (e == hipSuccess) e = hipEventRecord(aux->ev_aux[kb & 1], aux->stream);
        // A(kb) writes row block kb+1, which B(kb-1) writes too
        if (e == hipSuccess && kb > 0) e = hipStreamWaitEvent(st, aux->ev_aux[(kb - 1) & 1], 0);
        // A(kb) on st: row block kb+1 (columns outside block kb), then column
        // block kb+1 (rows outside blocks kb, kb+1).  A(kb), pivot(kb+1) and
        // panels(kb+1) are the critical path: their waves run at a raised
        // priority, so that the SIMDs they share with B(kb) issue their
        // instructions first.
        const Rect qa{rl1, rh1, rh1, rh1, 0, p.ncc, cl, ch};
        const Rect qb{0, p.nrc, rl, rh1, cl1, ch1, ch1, ch1};
        const double ua = bs1 * ((double)D - bs) * bs, ub = rest2 * bs1 * bs;
        // the K-split form where the chain is the critical path (measured: D =
        // 2048 2.49 -> 1.50 ms, 4096 5.03 -> 3.50, 6144 8.74 -> 8.26); at 8192
        // the bulk update hides the chain and the split waves only add
        // contention (17.14 -> 17.29 ms)
        if (split) {
            if (e == hipSuccess) e = lookahead_s<S8>(p, T, ld, kb, qa, qb, ua + ub, st);
        } else {
            if (e == hipSuccess) e = update_rect<S8>(p, T, ld, kb, qa, st, ua, true);
            if (e == hipSuccess) e = update_rect<S8>(p, T, ld, kb, qb, st, ub, true);
        }
        if (e == hipSuccess) e = pivot_s<S8>(T, ld, D, kb + 1, st);
        if (e == hipSuccess)
            e = split ? panels_split_s<S8>(p, T, ld, kb + 1, st)
                      : panels_s<S8>(T, ld, D, kb + 1, st);
        if (e != hipSuccess) break;
    }
    if (aux) aux_release(aux);
    return e;
}

}  // namespace

hipError_t launch_ad_mul(bool s8, uint16_t *C, int64_t ldc, const uint16_t *A, int64_t lda,
                         const uint16_t *B, int64_t ldb, int64_t R, int64_t K, int64_t N,
                         bool accumulate, hipStream_t stream, int64_t bspan,
                         const int *gate, const uint16_t *prev, int *flag) {
    const int64_t bmax = bspan >= 0 ? bspan : ldb;
    if (!flag) prev = nullptr;
    return s8 ? mul_s<true>(C, ldc, A, lda, B, ldb, R, K, N, accumulate, bmax, gate, prev, flag,
                            stream)
              : mul_s<false>(C, ldc, A, lda, B, ldb, R, K, N, accumulate, bmax, gate, prev, flag,
                             stream);
}

hipError_t launch_ad_mul_group(bool s8, const MulDesc *d, int n, bool accumulate,
                               hipStream_t stream) {
    return s8 ? mul_group_s<true>(d, n, accumulate, stream)
              : mul_group_s<false>(d, n, accumulate, stream);
}

hipError_t launch_ad_closure(bool s8, uint16_t *T, int64_t ld, int64_t D, bool serial,
                             hipStream_t stream, bool aux_create) {
    return s8 ? closure_s<true>(T, ld, D, serial, stream, aux_create)
              : closure_s<false>(T, ld, D, serial, stream, aux_create);
}

hipError_t launch_ad_fw_pivot(bool s8, uint16_t *T, int64_t ld, int64_t D, int64_t kb,
                              hipStream_t stream) {
    return s8 ? pivot_s<true>(T, ld, D, kb, stream) : pivot_s<false>(T, ld, D, kb, stream);
}

hipError_t launch_ad_fw_panels(bool s8, uint16_t *T, int64_t ld, int64_t D, int64_t kb,
                               hipStream_t stream) {
    return s8 ? panels_s<true>(T, ld, D, kb, stream) : panels_s<false>(T, ld, D, kb, stream);
}

hipError_t launch_ad_fw_update(bool s8, uint16_t *T, int64_t ld, int64_t D, int64_t kb,
                               hipStream_t stream) {
    const Plan p = make_plan(D);
    int rl, rh, cl, ch;
    block_chunks(D, kb, p.rw, &rl, &rh);
    block_chunks(D, kb, p.cw, &cl, &ch);
    const Rect q{0, p.nrc, rl, rh, 0, p.ncc, cl, ch};
    const double bs = block_bs(D, kb), rest = (double)D - bs;
    return s8 ? update_rect<true>(p, T, ld, kb, q, stream, rest * rest * bs)
              : update_rect<false>(p, T, ld, kb, q, stream, rest * rest * bs);
}

hipError_t launch_widen_u8(uint16_t *dst, int64_t ldd, const uint8_t *src, int64_t lds, int64_t R,
                           int64_t C, hipStream_t stream) {
    const int64_t n = R * ((C + 7) / 8);
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_widen, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, dst, ldd,
                       src, lds, R, C);
    return hipGetLastError();
}

hipError_t launch_narrow_u8(uint8_t *dst, int64_t ldd, const uint16_t *src, int64_t lds, int64_t R,
                            int64_t C, hipStream_t stream) {
    const int64_t n = R * ((C + 7) / 8);
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_narrow, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, dst, ldd,
                       src, lds, R, C);
    return hipGetLastError();
}

}  // namespace sr
