// Boolean semiring product and blocked Warshall closure on bit-packed
// matrices (Sec. II; bit layout of the paper's Boolean listing, Sec. IV:
// entry (r, c) is bit c % 64 of 64-bit word c / 64 of row r, so bit c % 32 of
// 32-bit word c / 32 on this little-endian device).
//
// Product: for each k, every row i with A_ik = 1 takes the OR of row k of B
// (the column-times-row sum of Sec. II).  A wavefront owns 64 rows (one per
// lane) and 32*NWB columns; row k of B is the same for all lanes, so its words
// are read with scalar loads, and each lane turns its bit A_ik into an
// all-ones / all-zeros mask.  The update of 32 entries is one v_and_or_b32:
// acc = (B_k & mask) | acc.
//
// Closure: Warshall's loop blocked in rounds of kBoolBlock pivots, with the
// same three phases as the anti-distance closure (pivot tile, panels, rest).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <stdlib.h>

#include <algorithm>

#include "sr_internal.h"

namespace sr {
namespace {

// Rows of B are read through the constant address space so that the
// compiler reads these wave-uniform rows with scalar loads (see sr_tiles.h);
// a row a kernel also writes is only ever re-read with the same bits.
#define kconst __attribute__((address_space(4)))

// One wavefront: rows [0, nrows) of a tile (lane = row), output 32-bit words
// [0, nw) with nw <= NWB, C (|)= A * B over K inner bits.  Strides in 32-bit
// words.  B rows are always read as whole NWB-word segments (the caller
// guarantees they fit in the padded rows); words >= nw feed only accumulators
// that are not stored.  A's bits at inner indices >= K inside the last word
// read are never used.  FULL: nw == NWB.  Lanes >= nrows compute on row 0 and
// store nothing.
template <int NWB, bool FULL, bool GROUPB = false>
__device__ __forceinline__ void bool_tile_body(uint32_t *C, int64_t ldc, const uint32_t *A,
                                               int64_t lda, const uint32_t *B, int64_t ldb,
                                               int nrows, int nw, int K, bool accumulate,
                                               bool sync_before_store) {
    static_assert(NWB % 4 == 0, "NWB must be a multiple of 4");
    const int lane = threadIdx.x & 63;
    const bool live = lane < nrows;
    const int64_t r = live ? lane : 0;
    uint32_t acc[NWB];
    uint32_t *crow = C + r * ldc;
    if (accumulate) {
        if (FULL) {
#pragma unroll
            for (int q = 0; q < NWB / 4; q++) {
                const uint4 v = reinterpret_cast<const uint4 *>(crow)[q];
                acc[4 * q] = v.x;
                acc[4 * q + 1] = v.y;
                acc[4 * q + 2] = v.z;
                acc[4 * q + 3] = v.w;
            }
        } else {
#pragma unroll
            for (int w = 0; w < NWB; w++) acc[w] = (w < nw) ? crow[w] : 0u;
        }
    } else {
#pragma unroll
        for (int w = 0; w < NWB; w++) acc[w] = 0u;
    }

    // KU inner bits per iteration: their KU rows of B occupy KU * NWB = 64
    // SGPRs.  Per row of B: one v_bfe_i32 turns bit k of the lane's A word
    // into a 0 / all-ones mask, then one v_bitop3_b32 per word computes
    // (B_k & mask) | acc (truth table 0xEA over src0 = B, src1 = mask,
    // src2 = acc), which the compiler cannot re-associate into AND + OR3.
    constexpr int KU = NWB >= 32 ? 2 : (NWB >= 16 ? 4 : 8);
    const uint32_t *arow = A + r * lda;
    int k = 0;
    if (K >= 32) {
        uint32_t anext = arow[0];
        for (; k + 32 <= K; k += 32) {
            const uint32_t a = anext;
            if (k + 64 <= K) anext = arow[(k >> 5) + 1];
#pragma unroll 1
            for (int g = 0; g < 32; g += KU) {
                const uint32_t *b0 = B + (int64_t)(k + g) * ldb;
                // with GROUPB the KU rows are loaded before the first update
                // (one wait per group: the square of a sparse 256-vertex
                // graph 26 -> 23 us; the closures' update kernels,
                // with many waves in flight, do not gain and keep per-row loads)
                uint32_t bg[GROUPB ? KU : 1][NWB];
                if constexpr (GROUPB) {
#pragma unroll
                    for (int u = 0; u < KU; u++) {
                        const kconst uint32_t *bp = (const kconst uint32_t *)(b0 + u * ldb);
#pragma unroll
                        for (int w = 0; w < NWB; w++) bg[u][w] = bp[w];
                    }
                }
#pragma unroll
                for (int u = 0; u < KU; u++) {
                    const uint32_t m = (uint32_t)__builtin_amdgcn_sbfe(a, g + u, 1);
                    const kconst uint32_t *brow = (const kconst uint32_t *)(b0 + u * ldb);
#pragma unroll
                    for (int w = 0; w < NWB; w++)
                        acc[w] = __builtin_amdgcn_bitop3_b32(GROUPB ? bg[u][w] : brow[w], m,
                                                             acc[w], 0xEA);
                }
            }
        }
    }
    if (k < K) {
        const uint32_t a = arow[k >> 5];
        for (int b = 0; k + b < K; b++) {
            const uint32_t m = (uint32_t)__builtin_amdgcn_sbfe(a, b, 1);
            const kconst uint32_t *brow = (const kconst uint32_t *)(B + (int64_t)(k + b) * ldb);
#pragma unroll
            for (int w = 0; w < NWB; w++)
                acc[w] = __builtin_amdgcn_bitop3_b32(brow[w], m, acc[w], 0xEA);
        }
    }

    if (sync_before_store) __syncthreads();
    if (!live) return;
    if (FULL) {
#pragma unroll
        for (int q = 0; q < NWB / 4; q++)
            reinterpret_cast<uint4 *>(crow)[q] =
                uint4{acc[4 * q], acc[4 * q + 1], acc[4 * q + 2], acc[4 * q + 3]};
    } else {
#pragma unroll
        for (int w = 0; w < NWB; w++)
            if (w < nw) crow[w] = acc[w];
    }
}

// bspan: 32-bit words of each B row readable from the tile origin.  When a
// whole NWB-word segment fits, one NWB-wide tile; otherwise (the last chunk of
// a row whose length is not a multiple of NWB) 4-word tiles, whose 16-byte
// segments always fit because rows are padded to 16 bytes.  With
// sync_before_store the whole workgroup calls this (one barrier); in the
// 4-word fallback sub-tiles store as they finish and the barrier comes last,
// which is exact for the panel updates because the pivot tile is closed.
template <int NWB, bool GROUPB = false>
__device__ __forceinline__ void bool_tile(uint32_t *C, int64_t ldc, const uint32_t *A, int64_t lda,
                                          const uint32_t *B, int64_t ldb, int nrows, int nw,
                                          int64_t bspan, int K, bool accumulate,
                                          bool sync_before_store) {
    if (nrows <= 0 || nw <= 0) {
        if (sync_before_store) __syncthreads();
        return;
    }
    if (bspan >= NWB) {
        if (nw >= NWB)
            bool_tile_body<NWB, true, GROUPB>(C, ldc, A, lda, B, ldb, nrows, NWB, K, accumulate,
                                              sync_before_store);
        else
            bool_tile_body<NWB, false, GROUPB>(C, ldc, A, lda, B, ldb, nrows, nw, K, accumulate,
                                               sync_before_store);
        return;
    }
    for (int c = 0; c < nw; c += 4) {
        const int n = min(4, nw - c);
        if (n == 4)
            bool_tile_body<4, true, GROUPB>(C + c, ldc, A, lda, B + c, ldb, nrows, 4, K,
                                            accumulate, false);
        else
            bool_tile_body<4, false, GROUPB>(C + c, ldc, A, lda, B + c, ldb, nrows, n, K,
                                             accumulate, false);
    }
    if (sync_before_store) __syncthreads();
}

// Products with few output tiles and a long inner dimension (a 256 x 256 x
// 256 product has four 64-row x 8-word tiles): a workgroup of KS
// waves per tile, wave s taking a slice of the inner bits (a multiple of 8),
// so that each wave runs KS times fewer dependent steps.  The waves' partial
// rows are ORed together in LDS (exact in any order) and stored by the
// workgroup: thread t < 64 * 8 owns word t % 8 of the tile's row t / 8.
// Every B row segment read is 8 words from the tile's first word (the
// launcher checks that the padded rows hold them).
template <int KS>
__global__ void __launch_bounds__(64 * KS)
k_bool_mul_ksplit(uint32_t *C, int64_t ldc, const uint32_t *A, int64_t lda, const uint32_t *B,
                  int64_t ldb, int64_t R, int K, int64_t nwords, int accumulate) {
    constexpr int NWB = 8;
    __shared__ uint32_t part[KS][64][NWB];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int64_t row0 = (int64_t)blockIdx.y * 64, w0 = (int64_t)blockIdx.x * NWB;
    const int nrows = (int)min<int64_t>(64, R - row0);
    const int nw = (int)min<int64_t>(NWB, nwords - w0);
    const int64_t r = lane < nrows ? lane : 0;
    const uint32_t *arow = A + (row0 + r) * lda;
    const int kc = ((K + KS - 1) / KS + 7) & ~7;
    const int k0 = wave * kc, k1 = min(K, k0 + kc);
    uint32_t acc[NWB];
#pragma unroll
    for (int w = 0; w < NWB; w++) acc[w] = 0u;
    for (int k = k0; k < k1; k += 8) {
        const uint32_t a = arow[k >> 5];
        const uint32_t *b0 = B + (int64_t)k * ldb + w0;
        if (k + 8 <= k1) {
            // the group's eight rows of B loaded before its updates
            uint32_t bg[8][NWB];
#pragma unroll
            for (int u = 0; u < 8; u++) {
                const kconst uint32_t *bp = (const kconst uint32_t *)(b0 + u * ldb);
#pragma unroll
                for (int w = 0; w < NWB; w++) bg[u][w] = bp[w];
            }
#pragma unroll
            for (int u = 0; u < 8; u++) {
                const uint32_t m = (uint32_t)__builtin_amdgcn_sbfe(a, (k & 31) + u, 1);
#pragma unroll
                for (int w = 0; w < NWB; w++)
                    acc[w] = __builtin_amdgcn_bitop3_b32(bg[u][w], m, acc[w], 0xEA);
            }
        } else {
            for (int u = 0; k + u < k1; u++) {
                const uint32_t m = (uint32_t)__builtin_amdgcn_sbfe(a, (k & 31) + u, 1);
                const kconst uint32_t *bp = (const kconst uint32_t *)(b0 + u * ldb);
#pragma unroll
                for (int w = 0; w < NWB; w++)
                    acc[w] = __builtin_amdgcn_bitop3_b32(bp[w], m, acc[w], 0xEA);
            }
        }
    }
    reinterpret_cast<uint4 *>(part[wave][lane])[0] = uint4{acc[0], acc[1], acc[2], acc[3]};
    reinterpret_cast<uint4 *>(part[wave][lane])[1] = uint4{acc[4], acc[5], acc[6], acc[7]};
    __syncthreads();
    const int t = threadIdx.x;
    if (t >= 64 * NWB) return;
    const int row = t / NWB, w = t % NWB;
    uint32_t v = 0;
#pragma unroll
    for (int q = 0; q < KS; q++) v |= part[q][row][w];
    if (row < nrows && w < nw) {
        uint32_t *c = C + (row0 + row) * ldc + w0 + w;
        *c = accumulate ? (*c | v) : v;
    }
}

template <int NWB>
__global__ void __launch_bounds__(256)
k_bool_mul(uint32_t *C, int64_t ldc, const uint32_t *A, int64_t lda, const uint32_t *B, int64_t ldb,
           int64_t R, int K, int64_t nwords, int accumulate) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform per wave
    const int64_t row0 = ((int64_t)blockIdx.y * 4 + wave) * 64;
    const int64_t w0 = (int64_t)blockIdx.x * NWB;
    if (row0 >= R) return;
    bool_tile<NWB, true>(C + row0 * ldc + w0, ldc, A + row0 * lda, lda, B + w0, ldb,
                         (int)min<int64_t>(64, R - row0), (int)min<int64_t>(NWB, nwords - w0),
                         ldb - w0, K, accumulate != 0, false);
}

// Warshall step k = 64P + 32h + b of the pivot-tile closure, on the two
// words (d0, d1) of the calling wave's 64 rows that hold the columns of block
// P (row k is in lane 32h + b, read with v_readlane): rows with bit k set OR
// in those two words of row k.
__device__ __forceinline__ void diag_step(uint32_t &d0, uint32_t &d1, int h, int b) {
    const int src = 32 * h + b;
    const uint32_t m = (uint32_t)__builtin_amdgcn_sbfe(h ? d1 : d0, b, 1);
    const uint32_t x0 = __builtin_amdgcn_readlane(d0, src);
    const uint32_t x1 = __builtin_amdgcn_readlane(d1, src);
    d0 = __builtin_amdgcn_bitop3_b32(x0, m, d0, 0xEA);
    d1 = __builtin_amdgcn_bitop3_b32(x1, m, d1, 0xEA);
}

// LDS of the pivot-tile closure: block P's rows before the phase (orig), its
// 64 x 64 diagonal block closed (cw), and its rows after the phase (fin, two
// buffers used by alternate phases).
struct PivotLds {
    uint32_t orig[64][8];
    uint32_t fin[2][64][8];
    uint32_t cw[64][2];
};

// One 64-pivot phase of the pivot-tile closure (see k_bool_fw_pivot); P is
// the phase, so the words holding its pivot bits are registers known at
// compile time.  For the rows i of block P, Warshall's steps over the pivots
// k of the block give T'_ij = T_ij | OR_k C_ik & T_kj, with C the closure of
// the block's 64 x 64 diagonal block (paths whose inner vertices lie in the
// block) and T the rows before the phase: so only C is computed step by step
// (two words per row), and the other six words are that product.  The rows
// of the other blocks then take T'_ij = T_ij | OR_k T_ik & T'_kj (k in the
// block, T_ik before the phase), the block's final rows applied once each in
// any order.
//   1. wave P publishes its rows (orig) and closes its two diagonal words
//      step by step (5 instructions per step instead of 17 for all eight
//      words), then publishes them (cw, and as the diagonal words of fin);
//   2. after a barrier, wave q != P forms words 2q and 2q + 1 of block P's
//      rows as the product above (lane = row, row k of orig read by all lanes
//      at one address);
//   3. after a barrier, wave P takes its rows from fin and every other wave
//      applies fin to its own rows.
// Wave P + 1 rewrites orig and cw in the next phase only after passing this
// phase's second barrier, when every wave has finished reading them (step 3
// reads neither).  fin alternates between two buffers: the next phase writes
// the other one while slower waves may still read this one in step 3, and the
// phase after it writes this one only once every wave has passed the next
// phase's barriers, i.e. has finished step 3 here.
template <int P, bool PIPE>
__device__ __forceinline__ void pivot_phase(uint32_t (&r)[8], int wave, int lane, int bs,
                                            PivotLds &L) {
    const int kn = min(64, bs - 64 * P);
    if (kn <= 0) return;  // bs is uniform over the workgroup
    uint32_t (*fin)[8] = L.fin[P & 1];
    if (wave == P) {
        reinterpret_cast<uint4 *>(L.orig[lane])[0] = uint4{r[0], r[1], r[2], r[3]};
        reinterpret_cast<uint4 *>(L.orig[lane])[1] = uint4{r[4], r[5], r[6], r[7]};
        // the steps of a full half of 32 unrolled: the lane of row k is then
        // a constant, and a step's readlanes issue as soon as its words are
        // ready
#pragma unroll
        for (int h = 0; h < 2; h++) {
            const int n = min(32, kn - 32 * h);
            if (n == 32) {
#pragma unroll
                for (int b = 0; b < 32; b++) diag_step(r[2 * P], r[2 * P + 1], h, b);
            } else {
                for (int b = 0; b < n; b++) diag_step(r[2 * P], r[2 * P + 1], h, b);
            }
        }
        L.cw[lane][0] = r[2 * P];
        L.cw[lane][1] = r[2 * P + 1];
        fin[lane][2 * P] = r[2 * P];
        fin[lane][2 * P + 1] = r[2 * P + 1];
    }
    __syncthreads();
    if (wave != P) {
        const uint32_t c0 = L.cw[lane][0], c1 = L.cw[lane][1];
        uint32_t a0 = L.orig[lane][2 * wave], a1 = L.orig[lane][2 * wave + 1];
        const auto step = [&](uint32_t c, int k) __attribute__((always_inline)) {
            const uint32_t m = (uint32_t)__builtin_amdgcn_sbfe(c, k & 31, 1);
            const uint2 x = *reinterpret_cast<const uint2 *>(&L.orig[k][2 * wave]);
            a0 = __builtin_amdgcn_bitop3_b32(x.x, m, a0, 0xEA);
            a1 = __builtin_amdgcn_bitop3_b32(x.y, m, a1, 0xEA);
        };
#pragma unroll
        for (int h = 0; h < 2; h++) {
            const int n = min(32, kn - 32 * h);
            const uint32_t c = h ? c1 : c0;
            if (PIPE && n == 32) {
                // groups of 8 rows, the next group's LDS reads issued before
                // this group's updates (at most 15 LDS reads may be in flight)
                uint2 cur[8], nxt[8];
#pragma unroll
                for (int i = 0; i < 8; i++)
                    cur[i] = *reinterpret_cast<const uint2 *>(&L.orig[32 * h + i][2 * wave]);
#pragma unroll
                for (int g = 0; g < 4; g++) {
                    if (g < 3) {
#pragma unroll
                        for (int i = 0; i < 8; i++)
                            nxt[i] = *reinterpret_cast<const uint2 *>(
                                &L.orig[32 * h + 8 * (g + 1) + i][2 * wave]);
                    }
#pragma unroll
                    for (int i = 0; i < 8; i++) {
                        const uint32_t m = (uint32_t)__builtin_amdgcn_sbfe(c, 8 * g + i, 1);
                        a0 = __builtin_amdgcn_bitop3_b32(cur[i].x, m, a0, 0xEA);
                        a1 = __builtin_amdgcn_bitop3_b32(cur[i].y, m, a1, 0xEA);
                    }
                    if (g < 3) {
#pragma unroll
                        for (int i = 0; i < 8; i++) cur[i] = nxt[i];
                    }
                }
            } else {
                for (int b = 0; b < n; b++) step(c, 32 * h + b);
            }
        }
        fin[lane][2 * wave] = a0;
        fin[lane][2 * wave + 1] = a1;
    }
    __syncthreads();
    if (wave == P) {
        const uint4 f0 = reinterpret_cast<const uint4 *>(fin[lane])[0];
        const uint4 f1 = reinterpret_cast<const uint4 *>(fin[lane])[1];
        r[0] = f0.x, r[1] = f0.y, r[2] = f0.z, r[3] = f0.w;
        r[4] = f1.x, r[5] = f1.y, r[6] = f1.z, r[7] = f1.w;
    } else {
        // the masks are this row's bits of block P as they were before the
        // phase
        const uint32_t a0 = r[2 * P], a1 = r[2 * P + 1];
        const auto step = [&](uint32_t a, int k) __attribute__((always_inline)) {
            const uint32_t m = (uint32_t)__builtin_amdgcn_sbfe(a, k & 31, 1);
            const uint4 p0 = reinterpret_cast<const uint4 *>(fin[k])[0];
            const uint4 p1 = reinterpret_cast<const uint4 *>(fin[k])[1];
            r[0] = __builtin_amdgcn_bitop3_b32(p0.x, m, r[0], 0xEA);
            r[1] = __builtin_amdgcn_bitop3_b32(p0.y, m, r[1], 0xEA);
            r[2] = __builtin_amdgcn_bitop3_b32(p0.z, m, r[2], 0xEA);
            r[3] = __builtin_amdgcn_bitop3_b32(p0.w, m, r[3], 0xEA);
            r[4] = __builtin_amdgcn_bitop3_b32(p1.x, m, r[4], 0xEA);
            r[5] = __builtin_amdgcn_bitop3_b32(p1.y, m, r[5], 0xEA);
            r[6] = __builtin_amdgcn_bitop3_b32(p1.z, m, r[6], 0xEA);
            r[7] = __builtin_amdgcn_bitop3_b32(p1.w, m, r[7], 0xEA);
        };
#pragma unroll
        for (int h = 0; h < 2; h++) {
            const int n = min(32, kn - 32 * h);
            const uint32_t a = h ? a1 : a0;
            if (PIPE && n == 32) {
                // groups of 4 rows (8 LDS reads), the next group's reads
                // issued before this group's updates
                uint4 cur[4][2], nxt[4][2];
#pragma unroll
                for (int i = 0; i < 4; i++) {
                    cur[i][0] = reinterpret_cast<const uint4 *>(fin[32 * h + i])[0];
                    cur[i][1] = reinterpret_cast<const uint4 *>(fin[32 * h + i])[1];
                }
#pragma unroll
                for (int g = 0; g < 8; g++) {
                    if (g < 7) {
#pragma unroll
                        for (int i = 0; i < 4; i++) {
                            nxt[i][0] = reinterpret_cast<const uint4 *>(fin[32 * h + 4 * (g + 1) + i])[0];
                            nxt[i][1] = reinterpret_cast<const uint4 *>(fin[32 * h + 4 * (g + 1) + i])[1];
                        }
                    }
#pragma unroll
                    for (int i = 0; i < 4; i++) {
                        const uint32_t m = (uint32_t)__builtin_amdgcn_sbfe(a, 4 * g + i, 1);
                        const uint4 p0 = cur[i][0], p1 = cur[i][1];
                        r[0] = __builtin_amdgcn_bitop3_b32(p0.x, m, r[0], 0xEA);
                        r[1] = __builtin_amdgcn_bitop3_b32(p0.y, m, r[1], 0xEA);
                        r[2] = __builtin_amdgcn_bitop3_b32(p0.z, m, r[2], 0xEA);
                        r[3] = __builtin_amdgcn_bitop3_b32(p0.w, m, r[3], 0xEA);
                        r[4] = __builtin_amdgcn_bitop3_b32(p1.x, m, r[4], 0xEA);
                        r[5] = __builtin_amdgcn_bitop3_b32(p1.y, m, r[5], 0xEA);
                        r[6] = __builtin_amdgcn_bitop3_b32(p1.z, m, r[6], 0xEA);
                        r[7] = __builtin_amdgcn_bitop3_b32(p1.w, m, r[7], 0xEA);
                    }
                    if (g < 7) {
#pragma unroll
                        for (int i = 0; i < 4; i++) {
                            cur[i][0] = nxt[i][0];
                            cur[i][1] = nxt[i][1];
                        }
                    }
                }
            } else {
                for (int b = 0; b < n; b++) step(a, 32 * h + b);
            }
        }
    }
}

// Pivot tile closure (bs <= 256): thread t holds row t of the tile as 8 words,
// wave p rows [64p, 64p + 64); Warshall's loop in four phases of 64 pivots
// (pivot_phase).  nwv: valid words of a tile row.  PIPE: the LDS reads of the
// product and apply steps are issued a group ahead (a tile alone on the
// device: 18.5 -> 17.0 us; beside the blocked closure's bulk update, where
// its larger register footprint costs more than it saves, off).
template <bool PIPE>
__global__ void __launch_bounds__(256)
k_bool_fw_pivot(uint32_t *T, int64_t ld, int64_t k0, int bs, int nwv, int prio) {
    if (prio) __builtin_amdgcn_s_setprio(2);
    __shared__ PivotLds lds;
    uint32_t *tile = T + k0 * ld + (k0 >> 5);
    const int t = threadIdx.x, lane = t & 63;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);  // uniform per wave
    const bool live = t < bs;
    uint32_t r[8];
    // rows are 16-byte aligned (base and stride), and the tile starts at a
    // multiple of 8 words: a whole row of 8 words moves as two 16-byte words
    uint32_t *row = tile + (int64_t)t * ld;
    if (live && nwv == 8) {
        const uint4 v0 = reinterpret_cast<const uint4 *>(row)[0];
        const uint4 v1 = reinterpret_cast<const uint4 *>(row)[1];
        r[0] = v0.x, r[1] = v0.y, r[2] = v0.z, r[3] = v0.w;
        r[4] = v1.x, r[5] = v1.y, r[6] = v1.z, r[7] = v1.w;
    } else {
#pragma unroll
        for (int j = 0; j < 8; j++) r[j] = (live && j < nwv) ? row[j] : 0u;
    }
    pivot_phase<0, PIPE>(r, wave, lane, bs, lds);
    pivot_phase<1, PIPE>(r, wave, lane, bs, lds);
    pivot_phase<2, PIPE>(r, wave, lane, bs, lds);
    pivot_phase<3, PIPE>(r, wave, lane, bs, lds);
    if (!live) return;
    if (nwv == 8) {
        reinterpret_cast<uint4 *>(row)[0] = uint4{r[0], r[1], r[2], r[3]};
        reinterpret_cast<uint4 *>(row)[1] = uint4{r[4], r[5], r[6], r[7]};
    } else {
#pragma unroll
        for (int j = 0; j < 8; j++)
            if (j < nwv) row[j] = r[j];
    }
}

// An 8-word-wide tile with its B block staged in LDS: all 64 * 4 * KH threads
// of the workgroup call this (it has barriers); B (K <= 256 rows of 8 words,
// from the workgroup-uniform pointer B) is the same for every wave, and the
// four row groups of waves (wave % 4) each update their own 64-row tile C
// (|)= A * B (nrows <= 0: nothing).  KH = 2: the waves 4 .. 7 take the
// second half of the inner steps of the same tiles and hand their partial
// ORs to waves 0 .. 3 through LDS (`part`), which store; each wave then runs
// half the dependent steps.  The B block is copied before any wave stores,
// so C may overlap B (the row panel: the closed pivot tile makes the result
// independent of that order).  nw <= 8 output words; bspan: words of each B
// row readable from B.
template <int KH>
__device__ __forceinline__ void bool_tile8_lds(uint32_t *C, int64_t ldc, const uint32_t *A,
                                               int64_t lda, const uint32_t *B, int64_t ldb,
                                               int nrows, int nw, int64_t bspan, int K,
                                               uint4 (*lds)[2], uint4 (*part)[64][2] = nullptr) {
    const int t = threadIdx.x;
    if (t < K) {
        const uint32_t *brow = B + (int64_t)t * ldb;
        if (bspan >= 8) {
            lds[t][0] = reinterpret_cast<const uint4 *>(brow)[0];
            lds[t][1] = reinterpret_cast<const uint4 *>(brow)[1];
        } else {
            uint32_t v[8];
#pragma unroll
            for (int w = 0; w < 8; w++) v[w] = w < bspan ? brow[w] : 0u;
            lds[t][0] = uint4{v[0], v[1], v[2], v[3]};
            lds[t][1] = uint4{v[4], v[5], v[6], v[7]};
        }
    }
    __syncthreads();
    const int lane = t & 63;
    const int half = KH == 2 ? __builtin_amdgcn_readfirstlane(t >> 8) : 0;  // uniform per wave
    const int sub = (t >> 6) & 3;
    const bool work = nrows > 0 && nw > 0;
    const bool live = lane < nrows;
    const int64_t r = live ? lane : 0;
    uint32_t *crow = C + r * ldc;
    uint32_t acc[8] = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
    // inner steps [kb, ke) of this wave (the halves split at a word boundary)
    const int kh = KH == 2 ? min(K, (K + 63) / 64 * 32) : K;
    const int kb = half ? kh : 0, ke = half ? K : kh;
    if (work) {
        if (!half) {
            if (nw == 8) {
                const uint4 c0 = reinterpret_cast<const uint4 *>(crow)[0];
                const uint4 c1 = reinterpret_cast<const uint4 *>(crow)[1];
                acc[0] = c0.x, acc[1] = c0.y, acc[2] = c0.z, acc[3] = c0.w;
                acc[4] = c1.x, acc[5] = c1.y, acc[6] = c1.z, acc[7] = c1.w;
            } else {
#pragma unroll
                for (int w = 0; w < 8; w++) acc[w] = w < nw ? crow[w] : 0u;
            }
        }
        const uint32_t *arow = A + r * lda;
        for (int kw = kb; kw < ke; kw += 32) {
            const uint32_t a = arow[kw >> 5];
            const int n = min(32, ke - kw);
            if (n == 32) {
#pragma unroll
                for (int b = 0; b < 32; b++) {
                    const uint32_t m = (uint32_t)__builtin_amdgcn_sbfe(a, b, 1);
                    const uint4 p0 = lds[kw + b][0], p1 = lds[kw + b][1];
                    acc[0] = __builtin_amdgcn_bitop3_b32(p0.x, m, acc[0], 0xEA);
                    acc[1] = __builtin_amdgcn_bitop3_b32(p0.y, m, acc[1], 0xEA);
                    acc[2] = __builtin_amdgcn_bitop3_b32(p0.z, m, acc[2], 0xEA);
                    acc[3] = __builtin_amdgcn_bitop3_b32(p0.w, m, acc[3], 0xEA);
                    acc[4] = __builtin_amdgcn_bitop3_b32(p1.x, m, acc[4], 0xEA);
                    acc[5] = __builtin_amdgcn_bitop3_b32(p1.y, m, acc[5], 0xEA);
                    acc[6] = __builtin_amdgcn_bitop3_b32(p1.z, m, acc[6], 0xEA);
                    acc[7] = __builtin_amdgcn_bitop3_b32(p1.w, m, acc[7], 0xEA);
                }
            } else {
                for (int b = 0; b < n; b++) {
                    const uint32_t m = (uint32_t)__builtin_amdgcn_sbfe(a, b, 1);
                    const uint4 p0 = lds[kw + b][0], p1 = lds[kw + b][1];
                    acc[0] = __builtin_amdgcn_bitop3_b32(p0.x, m, acc[0], 0xEA);
                    acc[1] = __builtin_amdgcn_bitop3_b32(p0.y, m, acc[1], 0xEA);
                    acc[2] = __builtin_amdgcn_bitop3_b32(p0.z, m, acc[2], 0xEA);
                    acc[3] = __builtin_amdgcn_bitop3_b32(p0.w, m, acc[3], 0xEA);
                    acc[4] = __builtin_amdgcn_bitop3_b32(p1.x, m, acc[4], 0xEA);
                    acc[5] = __builtin_amdgcn_bitop3_b32(p1.y, m, acc[5], 0xEA);
                    acc[6] = __builtin_amdgcn_bitop3_b32(p1.z, m, acc[6], 0xEA);
                    acc[7] = __builtin_amdgcn_bitop3_b32(p1.w, m, acc[7], 0xEA);
                }
            }
        }
    }
    if constexpr (KH == 2) {
        if (half && work) {
            part[sub][lane][0] = uint4{acc[0], acc[1], acc[2], acc[3]};
            part[sub][lane][1] = uint4{acc[4], acc[5], acc[6], acc[7]};
        }
        __syncthreads();
        if (half || !work) return;
        const uint4 q0 = part[sub][lane][0], q1 = part[sub][lane][1];
        acc[0] |= q0.x, acc[1] |= q0.y, acc[2] |= q0.z, acc[3] |= q0.w;
        acc[4] |= q1.x, acc[5] |= q1.y, acc[6] |= q1.z, acc[7] |= q1.w;
    }
    if (!work || !live) return;
    if (nw == 8) {
        reinterpret_cast<uint4 *>(crow)[0] = uint4{acc[0], acc[1], acc[2], acc[3]};
        reinterpret_cast<uint4 *>(crow)[1] = uint4{acc[4], acc[5], acc[6], acc[7]};
    } else {
#pragma unroll
        for (int w = 0; w < 8; w++)
            if (w < nw) crow[w] = acc[w];
    }
}

// Phase 2.  Workgroups [0, n_rowwg): the 256 pivot rows (4 x 64) times one
// 8-word (256-column) chunk outside the pivot block.  The rest: column
// panel, 4 x 64 rows outside the pivot block times the 8 pivot words.
// Either way the workgroup shares one B block (the chunk's pivot rows, or
// the pivot tile), staged in LDS, and its eight waves split the inner steps
// in two halves (bool_tile8_lds<2>): the panels are on the critical path of
// the overlapped closure, where half-length dependent chains pay.
__global__ void __launch_bounds__(512)
k_bool_fw_panels(uint32_t *T, int64_t ld, int D, int k0, int bs, int n_rowwg, int prio) {
    if (prio) __builtin_amdgcn_s_setprio(2);
    __shared__ uint4 lds[256][2];
    __shared__ uint4 part[4][64][2];
    const int sub = __builtin_amdgcn_readfirstlane((threadIdx.x >> 6) & 3);  // row group
    const int64_t nwd = ((int64_t)D + 31) >> 5;
    const int kw0 = k0 >> 5;
    const int kpw = (int)min<int64_t>(8, nwd - kw0);
    if ((int)blockIdx.x < n_rowwg) {
        const int cc = (int)blockIdx.x;
        const int64_t c = cc < (kw0 >> 3) ? cc : cc + 1;
        const int64_t w0 = c * 8;
        const int rofs = sub * 64;
        const int64_t r0 = (int64_t)k0 + rofs;
        bool_tile8_lds<2>(T + r0 * ld + w0, ld, T + r0 * ld + kw0, ld, T + (int64_t)k0 * ld + w0,
                          ld, min(64, bs - rofs), (int)min<int64_t>(8, nwd - w0), ld - w0, bs, lds,
                          part);
    } else {
        const int kr0 = k0 / 64, kr1 = (k0 + bs + 63) / 64;
        const int rc = ((int)blockIdx.x - n_rowwg) * 4 + sub;
        const int rchunk = rc < kr0 ? rc : rc + (kr1 - kr0);
        const int64_t row0 = (int64_t)rchunk * 64;
        const int nrows = (int)min<int64_t>(64, (int64_t)D - row0);  // <= 0 past the end
        bool_tile8_lds<2>(T + row0 * ld + kw0, ld, T + row0 * ld + kw0, ld,
                          T + (int64_t)k0 * ld + kw0, ld, nrows, kpw, ld - kw0, bs, lds, part);
    }
}

// Phase 3 over a rectangle: 64-row chunks [r_lo, r_hi) minus [r_ex0, r_ex1),
// times the 32-bit words [w0a, w0b) and [w1a, w1b), each word range cut into
// chunks of NWB words (the last one may be partial); T_ij (|)= T_iK * T_Kj for
// the pivot block K = [k0, k0 + bs).  Workgroups [0, nch0) take chunks of the
// first word range; each of a workgroup's four waves takes one row chunk.
template <int NWB>
__global__ void __launch_bounds__(256)
k_bool_fw_update(uint32_t *T, int64_t ld, int D, int k0, int bs, BRect q, int nch0, int prio) {
    if (prio) __builtin_amdgcn_s_setprio(2);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform per wave
    int rc = q.r_lo + (int)blockIdx.y * 4 + wave;
    if (rc >= q.r_ex0) rc += q.r_ex1 - q.r_ex0;
    const int cx = (int)blockIdx.x;
    const int w0 = cx < nch0 ? q.w0a + cx * NWB : q.w1a + (cx - nch0) * NWB;
    const int wend = cx < nch0 ? q.w0b : q.w1b;
    const int64_t row0 = (int64_t)rc * 64;
    const int nrows = rc < q.r_hi ? (int)min<int64_t>(64, (int64_t)D - row0) : 0;
    const int nw = min(NWB, wend - w0);
    uint32_t *C = T + row0 * ld + w0;
    const uint32_t *A = T + row0 * ld + (k0 >> 5), *B = T + (int64_t)k0 * ld + w0;
    if constexpr (NWB == 8) {
        // narrow chunks (small matrices): the four waves share the chunk's B
        // block through LDS
        __shared__ uint4 lds[256][2];
        bool_tile8_lds<1>(C, ld, A, ld, B, ld, nrows, nw, ld - w0, bs, lds);
    } else {
        if (nrows <= 0) return;
        if (nw == NWB) {
            bool_tile<NWB>(C, ld, A, ld, B, ld, nrows, NWB, ld - w0, bs, true, false);
        } else {
            // the partial chunk at the end of a word range, as 8-word tiles,
            // so that its cost follows its width
            for (int c = 0; c < nw; c += 8)
                bool_tile<8>(C + c, ld, A, ld, B + c, ld, nrows, min(8, nw - c), ld - w0 - c, bs,
                             true, false);
        }
    }
}

// The lookahead part of a round's update, A(kb) = rectangles qa (row block
// kb+1) and qb (column block kb+1), in one launch with short waves: a
// workgroup owns one 64-row x 8-word tile and its four waves split the inner
// bits -- wave w takes pivots [64w, 64w + 64) -- so each wave runs a quarter
// of the steps.  Each wave stages its 64 rows of B in LDS; the four partial
// ORs are combined in LDS and OR-ed into C by one store per word.  Workgroups
// [0, nwg_a) take tiles of qa; tile index t -> word chunk t % nch, row chunk
// t / nch (with the rectangle's row exclusion).
struct LaTile {
    int rc, w0, nw;
};

__device__ __forceinline__ LaTile la_tile(const BRect &q, int t) {
    const int nch0 = q.w0b > q.w0a ? (q.w0b - q.w0a + 7) / 8 : 0;
    const int nch1 = q.w1b > q.w1a ? (q.w1b - q.w1a + 7) / 8 : 0;
    const int nch = nch0 + nch1;
    const int cx = t % nch;
    int rc = q.r_lo + t / nch;
    if (rc >= q.r_ex0) rc += q.r_ex1 - q.r_ex0;
    LaTile r;
    r.rc = rc;
    r.w0 = cx < nch0 ? q.w0a + cx * 8 : q.w1a + (cx - nch0) * 8;
    r.nw = min(8, (cx < nch0 ? q.w0b : q.w1b) - r.w0);
    return r;
}

__host__ __device__ inline int la_tiles(const BRect &q) {
    const int nch0 = q.w0b > q.w0a ? (q.w0b - q.w0a + 7) / 8 : 0;
    const int nch1 = q.w1b > q.w1a ? (q.w1b - q.w1a + 7) / 8 : 0;
    const int nrows = (q.r_hi - q.r_lo) - (q.r_ex1 - q.r_ex0);
    return nrows > 0 ? (nch0 + nch1) * nrows : 0;
}

__global__ void __launch_bounds__(256)
k_bool_fw_lookahead(uint32_t *T, int64_t ld, int D, int k0, int bs, BRect qa, BRect qb, int nwg_a,
                    int prio) {
    if (prio) __builtin_amdgcn_s_setprio(2);
    __shared__ uint4 bl[256][2];       // B rows (pivot rows), 8 words each
    __shared__ uint32_t red[4][8][64];  // partial ORs: wave, word, lane
    const int t = threadIdx.x, lane = t & 63;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);  // uniform per wave
    const int bid = (int)blockIdx.x;
    const LaTile tile = bid < nwg_a ? la_tile(qa, bid) : la_tile(qb, bid - nwg_a);
    const int64_t row0 = (int64_t)tile.rc * 64;
    const int nrows = (int)min<int64_t>(64, (int64_t)D - row0);
    const int64_t bspan = ld - tile.w0;
    // stage: thread t copies B row t (pivot row k0 + t), words [w0, w0 + 8)
    if (t < bs) {
        const uint32_t *brow = T + (int64_t)(k0 + t) * ld + tile.w0;
        if (bspan >= 8) {
            bl[t][0] = reinterpret_cast<const uint4 *>(brow)[0];
            bl[t][1] = reinterpret_cast<const uint4 *>(brow)[1];
        } else {
            uint32_t v[8];
#pragma unroll
            for (int w = 0; w < 8; w++) v[w] = w < bspan ? brow[w] : 0u;
            bl[t][0] = uint4{v[0], v[1], v[2], v[3]};
            bl[t][1] = uint4{v[4], v[5], v[6], v[7]};
        }
    }
    __syncthreads();
    const bool live = lane < nrows;
    const uint32_t *arow = T + (row0 + (live ? lane : 0)) * ld + (k0 >> 5) + 2 * wave;
    const int kb0 = 64 * wave;
    const int kn = min(64, bs - kb0);  // this wave's pivots (<= 0: none)
    uint32_t acc[8] = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
#pragma unroll
    for (int h = 0; h < 2; h++) {
        const int n = min(32, kn - 32 * h);
        if (n <= 0) break;
        const uint32_t a = arow[h];
        for (int b = 0; b < n; b++) {
            const uint32_t m = (uint32_t)__builtin_amdgcn_sbfe(a, b, 1);
            const uint4 p0 = bl[kb0 + 32 * h + b][0], p1 = bl[kb0 + 32 * h + b][1];
            acc[0] = __builtin_amdgcn_bitop3_b32(p0.x, m, acc[0], 0xEA);
            acc[1] = __builtin_amdgcn_bitop3_b32(p0.y, m, acc[1], 0xEA);
            acc[2] = __builtin_amdgcn_bitop3_b32(p0.z, m, acc[2], 0xEA);
            acc[3] = __builtin_amdgcn_bitop3_b32(p0.w, m, acc[3], 0xEA);
            acc[4] = __builtin_amdgcn_bitop3_b32(p1.x, m, acc[4], 0xEA);
            acc[5] = __builtin_amdgcn_bitop3_b32(p1.y, m, acc[5], 0xEA);
            acc[6] = __builtin_amdgcn_bitop3_b32(p1.z, m, acc[6], 0xEA);
            acc[7] = __builtin_amdgcn_bitop3_b32(p1.w, m, acc[7], 0xEA);
        }
    }
#pragma unroll
    for (int w = 0; w < 8; w++) red[wave][w][lane] = acc[w];
    __syncthreads();
    // wave w ORs words 2w, 2w+1 of the four partials into C
    if (!live) return;
#pragma unroll
    for (int j = 0; j < 2; j++) {
        const int w = 2 * wave + j;
        if (w < tile.nw) {
            uint32_t *c = T + (row0 + lane) * ld + tile.w0 + w;
            *c = *c | red[0][w][lane] | red[1][w][lane] | red[2][w][lane] | red[3][w][lane];
        }
    }
}

// "Four Russians" tile (the paper mentions the method for the product and
// leaves it out; here it serves the product and the closure's bulk update,
// whose operands do not change during the update): C (|)= A * B for 256 rows
// (thread t: row row0 + t) x kM4rWords words.  For each group of 8 inner
// bits g, the workgroup builds in LDS the table L_g[v] = OR of the rows
// 8g + b of B with bit b of v set (256 entries), then every row ORs in the
// single entry picked by its 8 bits of A: one table read per row and group
// instead of 8 masked ORs per word.  Table build: thread (p, w) = (t / 16,
// t % 16) forms the 16 ORs of rows 8g..8g+3 in registers, ORs in its subset
// p of rows 8g+4..8g+7 and writes entries 16p .. 16p + 15 of word w.  Two
// tables alternate, so one barrier per group suffices (a table is rewritten
// only after every thread has passed the next group's barrier).  Rows are
// padded to kM4rStride words so that the 16-byte reads of 64 random entries
// spread over the LDS banks.  K inner bits; rows >= K of B and bits >= K of A
// count as zero; nwords: valid words of a C row from w0.
constexpr int kM4rWords = 16, kM4rStride = 20;

// TR rows per thread: thread t takes rows t, t + 256, ... (TR * 256 rows).
// NT tables in LDS: 2 alternate (one barrier per group), 1 is rewritten after
// a second barrier (half the LDS, so that kernels running beside this one
// still find room).
template <int TR, int NT>
__device__ __forceinline__ void m4r_tile(uint32_t *C, int64_t ldc, const uint32_t *A, int64_t lda,
                                         const uint32_t *B, int64_t ldb, int nrows, int nw, int K,
                                         bool accumulate, uint32_t (*lut)[256][kM4rStride]) {
    constexpr int CN = kM4rWords;
    const int t = threadIdx.x;
    uint32_t acc[TR][CN];
    const uint32_t *arow[TR];
    uint32_t *crow[TR];
    bool live[TR];
#pragma unroll
    for (int u = 0; u < TR; u++) {
        live[u] = t + 256 * u < nrows;
        const int64_t r = live[u] ? t + 256 * u : 0;
        crow[u] = C + r * ldc;
        arow[u] = A + r * lda;
        if (accumulate && nw == CN) {
#pragma unroll
            for (int q = 0; q < CN / 4; q++) {
                const uint4 v = reinterpret_cast<const uint4 *>(crow[u])[q];
                acc[u][4 * q] = v.x, acc[u][4 * q + 1] = v.y;
                acc[u][4 * q + 2] = v.z, acc[u][4 * q + 3] = v.w;
            }
        } else {
#pragma unroll
            for (int w = 0; w < CN; w++) acc[u][w] = (accumulate && w < nw) ? crow[u][w] : 0u;
        }
    }
    // table-builder role of this thread
    const int bw = t & (CN - 1), bp = t >> 4;
    const bool wok = bw < nw;
    const int ngroups = (K + 7) >> 3;
    // the 8 words of B a group needs are requested one group ahead, and each
    // row's A word one word ahead, so that their latency overlaps work
    auto fetch_b = [&](uint32_t(&dst)[8], int g) {
#pragma unroll
        for (int j = 0; j < 8; j++) {
            const int k = 8 * g + j;
            dst[j] = (wok && k < K) ? B[(int64_t)k * ldb + bw] : 0u;
        }
    };
    uint32_t a[TR], an[TR], bn[8];
    fetch_b(bn, 0);
#pragma unroll
    for (int u = 0; u < TR; u++) an[u] = K > 0 ? arow[u][0] : 0u;  // A may be NULL when K = 0
    for (int g = 0; g < ngroups; g++) {
        uint32_t (*L)[kM4rStride] = lut[NT == 2 ? (g & 1) : 0];
        uint32_t b[8];
#pragma unroll
        for (int j = 0; j < 8; j++) b[j] = bn[j];
        if (g + 1 < ngroups) fetch_b(bn, g + 1);
        if ((g & 3) == 0) {
#pragma unroll
            for (int u = 0; u < TR; u++) {
                a[u] = an[u];
                if (8 * g + 32 < K) an[u] = arow[u][(g >> 2) + 1];
            }
        }
        __builtin_amdgcn_sched_barrier(0);
        if (NT == 1 && g > 0) __syncthreads();  // the previous group's reads are done
        uint32_t lo[16];
        lo[0] = 0u;
#pragma unroll
        for (int v = 1; v < 16; v++) lo[v] = lo[v & (v - 1)] | b[__builtin_ctz(v)];
        uint32_t hi = 0u;
#pragma unroll
        for (int j = 0; j < 4; j++) hi |= ((bp >> j) & 1) ? b[4 + j] : 0u;
#pragma unroll
        for (int v = 0; v < 16; v++) L[16 * bp + v][bw] = hi | lo[v];
        __syncthreads();
#pragma unroll
        for (int u = 0; u < TR; u++) {
            const uint32_t sel = (a[u] >> (8 * (g & 3))) & 0xFFu;
            const uint4 *e = reinterpret_cast<const uint4 *>(L[sel]);
#pragma unroll
            for (int q = 0; q < CN / 4; q++) {
                const uint4 v = e[q];
                acc[u][4 * q] |= v.x, acc[u][4 * q + 1] |= v.y;
                acc[u][4 * q + 2] |= v.z, acc[u][4 * q + 3] |= v.w;
            }
        }
    }
#pragma unroll
    for (int u = 0; u < TR; u++) {
        if (!live[u]) continue;
        if (nw == CN) {
#pragma unroll
            for (int q = 0; q < CN / 4; q++)
                reinterpret_cast<uint4 *>(crow[u])[q] =
                    uint4{acc[u][4 * q], acc[u][4 * q + 1], acc[u][4 * q + 2], acc[u][4 * q + 3]};
        } else {
#pragma unroll
            for (int w = 0; w < CN; w++)
                if (w < nw) crow[u][w] = acc[u][w];
        }
    }
}

// Product with the four-Russians tile: workgroup (x, y) = words
// [16x, 16x + 16) of rows [256 TR y, 256 TR (y + 1)).
template <int TR>
__global__ void __launch_bounds__(256)
k_bool_mul_m4r(uint32_t *C, int64_t ldc, const uint32_t *A, int64_t lda, const uint32_t *B,
               int64_t ldb, int64_t R, int K, int64_t nwords, int accumulate) {
    __shared__ __align__(16) uint32_t lut[2][256][kM4rStride];
    const int64_t row0 = (int64_t)blockIdx.y * 256 * TR, w0 = (int64_t)blockIdx.x * kM4rWords;
    m4r_tile<TR, 2>(C + row0 * ldc + w0, ldc, A + row0 * lda, lda, B + w0, ldb,
                 (int)min<int64_t>(256 * TR, R - row0), (int)min<int64_t>(kM4rWords, nwords - w0),
                 K, accumulate != 0, lut);
}

// Bulk update of a closure round with the four-Russians tile: rows
// [r0a, r0b) and [r1a, r1b), words [w0a, w0b) and [w1a, w1b), each range cut
// into tiles of 512 rows x 16 words from its start; T_ij (|)= T_iK * T_Kj for
// the pivot block K = [k0, k0 + bs).  The tables hold rows of the pivot block,
// which the update does not write, and each row's A bits are its pivot-block
// words, outside every tile it writes.
struct MRect {
    int r0a, r0b, r1a, r1b;
    int w0a, w0b, w1a, w1b;
};

__global__ void __launch_bounds__(256)
k_bool_fw_update_m4r(uint32_t *T, int64_t ld, int k0, int bs, MRect q, int nwch0, int nrch0,
                     int prio) {
    if (prio) __builtin_amdgcn_s_setprio(2);
    __shared__ __align__(16) uint32_t lut[1][256][kM4rStride];
    const int bx = (int)blockIdx.x, by = (int)blockIdx.y;
    const int w0 = bx < nwch0 ? q.w0a + bx * kM4rWords : q.w1a + (bx - nwch0) * kM4rWords;
    const int wend = bx < nwch0 ? q.w0b : q.w1b;
    const int r0 = by < nrch0 ? q.r0a + by * 512 : q.r1a + (by - nrch0) * 512;
    const int rend = by < nrch0 ? q.r0b : q.r1b;
    m4r_tile<2, 1>(T + (int64_t)r0 * ld + w0, ld, T + (int64_t)r0 * ld + (k0 >> 5), ld,
                T + (int64_t)k0 * ld + w0, ld, min(512, rend - r0), min(kM4rWords, wend - w0), bs,
                true, lut);
}

template <int NWB>
hipError_t mul_nwb(uint32_t *C, int64_t ldc, const uint32_t *A, int64_t lda, const uint32_t *B,
                   int64_t ldb, int64_t R, int64_t K, int64_t nwords, bool acc, hipStream_t st) {
    const dim3 grid((unsigned)((nwords + NWB - 1) / NWB), (unsigned)((R + 255) / 256));
    hipLaunchKernelGGL((k_bool_mul<NWB>), grid, dim3(256), 0, st, C, ldc, A, lda, B, ldb, R, (int)K,
                       nwords, acc ? 1 : 0);
    return hipGetLastError();
}

template <int NWB>
hipError_t update_nwb(uint32_t *T, int64_t ld, int D, int k0, int bs, const BRect &q, int prio,
                      hipStream_t st) {
    const int nch0 = q.w0b > q.w0a ? (q.w0b - q.w0a + NWB - 1) / NWB : 0;
    const int nch1 = q.w1b > q.w1a ? (q.w1b - q.w1a + NWB - 1) / NWB : 0;
    const int nrows = (q.r_hi - q.r_lo) - (q.r_ex1 - q.r_ex0);
    const dim3 grid((unsigned)(nch0 + nch1), (unsigned)((nrows + 3) / 4));
    if (grid.x == 0 || nrows <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_bool_fw_update<NWB>), grid, dim3(256), 0, st, T, ld, D, k0, bs, q, nch0,
                       prio);
    return hipGetLastError();
}

// Rows [lo, hi) of block kb in 64-row chunks, and its 32-bit words.
struct BBlock {
    int k0, bs, rl, rh, wl, wh;
};

BBlock bblock(int64_t D, int64_t kb) {
    BBlock b;
    b.k0 = (int)(kb * kBoolBlock);
    b.bs = (int)std::min<int64_t>(kBoolBlock, D - b.k0);
    b.rl = b.k0 / 64;
    b.rh = (b.k0 + b.bs + 63) / 64;
    b.wl = b.k0 / 32;
    b.wh = (b.k0 + b.bs + 31) / 32;
    return b;
}

// Wave priority of the critical-path kernels (pivot, panels and the
// lookahead part of the update): raised, unless SR_PRIO=0 (for tuning).
int crit_prio() {
    static const int on = [] {
        const char *v = getenv("SR_PRIO");
        return v ? (atoi(v) != 0 ? 1 : 0) : 1;
    }();
    return on;
}

hipError_t pivot_b(uint32_t *T, int64_t ld, int64_t D, int64_t kb, hipStream_t st) {
    const BBlock b = bblock(D, kb);
    const int64_t nwd = (D + 31) / 32;
    const int nwv = (int)std::min<int64_t>(8, nwd - b.wl);
    const bool prof = prof_on();
    if (prof) prof_begin(st);
    // a closure of one tile: the tile is alone on the device
    if (D <= kBoolBlock)
        hipLaunchKernelGGL(k_bool_fw_pivot<true>, dim3(1), dim3(256), 0, st, T, ld, (int64_t)b.k0,
                           b.bs, nwv, crit_prio());
    else
        hipLaunchKernelGGL(k_bool_fw_pivot<false>, dim3(1), dim3(256), 0, st, T, ld,
                           (int64_t)b.k0, b.bs, nwv, crit_prio());
    hipError_t e = hipGetLastError();
    if (prof) prof_end(st, 0, 0, (double)b.bs * b.bs * b.bs);
    return e;
}

hipError_t panels_b(uint32_t *T, int64_t ld, int64_t D, int64_t kb, hipStream_t st) {
    const BBlock b = bblock(D, kb);
    const int64_t nwd = (D + 31) / 32;
    const int64_t nrch = (D + 63) / 64;
    const int n_rowwg = (int)((nwd + 7) / 8 - 1);
    const int n_colwg = (int)((nrch - (b.rh - b.rl) + 3) / 4);
    const bool prof = prof_on();
    if (prof) prof_begin(st);
    hipLaunchKernelGGL(k_bool_fw_panels, dim3(n_rowwg + n_colwg), dim3(512), 0, st, T, ld, (int)D,
                       b.k0, b.bs, n_rowwg, crit_prio());
    hipError_t e = hipGetLastError();
    if (prof) prof_end(st, 0, 1, 2.0 * ((double)D - b.bs) * b.bs * b.bs);
    return e;
}

hipError_t update_m4r(uint32_t *T, int64_t ld, int64_t D, const BBlock &b, const BRect &q,
                      hipStream_t st) {
    // 64-row chunk ranges -> row ranges
    MRect m;
    m.r0a = 64 * q.r_lo;
    m.r0b = (int)std::min<int64_t>(64 * (int64_t)q.r_ex0, D);
    m.r1a = (int)std::min<int64_t>(64 * (int64_t)q.r_ex1, D);
    m.r1b = (int)std::min<int64_t>(64 * (int64_t)q.r_hi, D);
    m.w0a = q.w0a, m.w0b = q.w0b, m.w1a = q.w1a, m.w1b = q.w1b;
    const int nr0 = m.r0b > m.r0a ? (m.r0b - m.r0a + 511) / 512 : 0;
    const int nr1 = m.r1b > m.r1a ? (m.r1b - m.r1a + 511) / 512 : 0;
    const int nw0 = m.w0b > m.w0a ? (m.w0b - m.w0a + kM4rWords - 1) / kM4rWords : 0;
    const int nw1 = m.w1b > m.w1a ? (m.w1b - m.w1a + kM4rWords - 1) / kM4rWords : 0;
    if (nr0 + nr1 == 0 || nw0 + nw1 == 0) return hipSuccess;
    hipLaunchKernelGGL(k_bool_fw_update_m4r, dim3(nw0 + nw1, nr0 + nr1), dim3(256), 0, st, T, ld,
                       b.k0, b.bs, m, nw0, nr0, 0);
    return hipGetLastError();
}

// nwb: word-chunk width of the bit-sliced kernel, 0 for the four-Russians
// kernel, kUpdateMfma for the matrix cores (the pivot rows transposed into
// pt first, on the same stream).
constexpr int kUpdateMfma = -1;
hipError_t update_b(uint32_t *T, int64_t ld, int64_t D, int64_t kb, const BRect &q, int nwb,
                    double units, hipStream_t st, bool critical = false,
                    uint32_t *pt = nullptr, bool transposed = false) {
    const BBlock b = bblock(D, kb);
    const int prio = critical ? crit_prio() : 0;
    const bool prof = prof_on();
    hipError_t e = hipSuccess;
    if (nwb == kUpdateMfma) {
        // (transposed: pt already holds round kb's pivot rows)
        if (!transposed) e = launch_bool_pivot_transpose(pt, T, ld, D, b.k0, b.bs, st);
        if (prof) prof_begin(st);
        if (e == hipSuccess) e = launch_bool_fw_update_mfma(T, ld, D, b.k0, q, pt, st);
        if (prof) prof_end(st, 0, 2, units);
        return e;
    }
    if (prof) prof_begin(st);
    if (nwb == 0) {
        e = update_m4r(T, ld, D, b, q, st);
        if (prof) prof_end(st, 0, 2, units);
        return e;
    }
    switch (nwb) {
        case 32: e = update_nwb<32>(T, ld, (int)D, b.k0, b.bs, q, prio, st); break;
        case 16: e = update_nwb<16>(T, ld, (int)D, b.k0, b.bs, q, prio, st); break;
        default: e = update_nwb<8>(T, ld, (int)D, b.k0, b.bs, q, prio, st); break;
    }
    if (prof) prof_end(st, 0, 2, units);
    return e;
}

}  // namespace

hipError_t launch_bool_mul_m4r(uint64_t *C, int64_t ldc, const uint64_t *A, int64_t lda,
                               const uint64_t *B, int64_t ldb, int64_t R, int64_t K, int64_t N,
                               bool accumulate, hipStream_t stream) {
    const int64_t nwords = (N + 31) / 32;
    const dim3 grid((unsigned)((nwords + kM4rWords - 1) / kM4rWords), (unsigned)((R + 511) / 512));
    hipLaunchKernelGGL(k_bool_mul_m4r<2>, grid, dim3(256), 0, stream,
                       reinterpret_cast<uint32_t *>(C), 2 * ldc,
                       reinterpret_cast<const uint32_t *>(A), 2 * lda,
                       reinterpret_cast<const uint32_t *>(B), 2 * ldb, R, (int)K, nwords,
                       accumulate ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_bool_mul(uint64_t *C, int64_t ldc, const uint64_t *A, int64_t lda,
                           const uint64_t *B, int64_t ldb, int64_t R, int64_t K, int64_t N,
                           bool accumulate, int path, hipStream_t stream) {
    // the four-Russians tables win once their 512-row x 512-column tiles
    // give the device a few workgroups per compute unit and K is long enough
    // to amortise each table
    const int64_t tiles = ((R + 511) / 512) * ((N + 511) / 512);
    if (path == kBoolPathM4r || (path == kBoolPathAuto && tiles >= 256 && K >= 1024))
        return launch_bool_mul_m4r(C, ldc, A, lda, B, ldb, R, K, N, accumulate, stream);
    uint32_t *c = reinterpret_cast<uint32_t *>(C);
    const uint32_t *a = reinterpret_cast<const uint32_t *>(A);
    const uint32_t *b = reinterpret_cast<const uint32_t *>(B);
    const int64_t nwords = (N + 31) / 32;
    // few 64-row x 8-word output tiles and a long inner dimension: the
    // inner bits split over sixteen waves per tile (256 x 256 x 256: one
    // workgroup of four waves, 13.8 us, against four of sixteen waves,
    // 3.6 us)
    const int64_t tiles8 = ((R + 63) / 64) * ((nwords + 7) / 8);
    if (path != kBoolPathM4r && tiles8 <= 64 && K >= 128 && K <= INT32_MAX &&
        2 * ldb >= (nwords + 7) / 8 * 8) {
        const dim3 grid((unsigned)((nwords + 7) / 8), (unsigned)((R + 63) / 64));
        hipLaunchKernelGGL(k_bool_mul_ksplit<16>, grid, dim3(1024), 0, stream, c, 2 * ldc, a,
                           2 * lda, b, 2 * ldb, R, (int)K, nwords, accumulate ? 1 : 0);
        return hipGetLastError();
    }
    int nwb = 32;
    while (nwb > 8 && ((R + 63) / 64) * ((nwords + nwb - 1) / nwb) < 4096) nwb >>= 1;
    switch (nwb) {
        case 32: return mul_nwb<32>(c, 2 * ldc, a, 2 * lda, b, 2 * ldb, R, K, nwords, accumulate, stream);
        case 16: return mul_nwb<16>(c, 2 * ldc, a, 2 * lda, b, 2 * ldb, R, K, nwords, accumulate, stream);
        default: return mul_nwb<8>(c, 2 * ldc, a, 2 * lda, b, 2 * ldb, R, K, nwords, accumulate, stream);
    }
}

// Blocked Warshall with one round of lookahead, as for anti-distances: the
// update of round kb is split into A(kb) -- row block kb+1 and column block
// kb+1, which the pivot and panels of round kb+1 need -- on the caller's
// stream, and B(kb) -- everything else -- on a second stream, where it
// overlaps A(kb), pivot(kb+1) and panels(kb+1).  The writes of B(kb) and of
// round kb+1's pivot and panels are disjoint, and B(kb) reads only row and
// column block kb, which round kb+1 does not write.  B(kb) is queued behind
// B(kb-1) as soon as panels(kb) is done; the caller's stream waits for
// B(kb-1) only before A(kb), which writes rows B(kb-1) also writes.
hipError_t lookahead_b(uint32_t *T, int64_t ld, int64_t D, int64_t kb, const BRect &qa,
                       const BRect &qb, double units, hipStream_t st) {
    const BBlock b = bblock(D, kb);
    const int na = la_tiles(qa), nb = la_tiles(qb);
    if (na + nb == 0) return hipSuccess;
    const bool prof = prof_on();
    if (prof) prof_begin(st);
    hipLaunchKernelGGL(k_bool_fw_lookahead, dim3(na + nb), dim3(256), 0, st, T, ld, (int)D, b.k0,
                       b.bs, qa, qb, na, crit_prio());
    hipError_t e = hipGetLastError();
    if (prof) prof_end(st, 0, 2, units);
    return e;
}

// Words per wave in the bulk update: wider tiles need fewer scalar loads per
// update, narrower ones give more waves to hide their latency.  SR_BOOL_NWB
// (8, 16 or 32) overrides the choice, for tuning.
int bool_update_nwb(int64_t D) {
    static const int forced = [] {
        const char *v = getenv("SR_BOOL_NWB");
        const int n = v ? atoi(v) : 0;
        return (n == 8 || n == 16 || n == 32) ? n : 0;
    }();
    if (forced) return forced;
    return D >= 8192 ? 32 : (D >= 2048 ? 16 : 8);
}

hipError_t launch_bool_closure(uint64_t *T64, int64_t ld64, int64_t D, bool serial, int path,
                               hipStream_t st, bool aux_create, void *work) {
    uint32_t *T = reinterpret_cast<uint32_t *>(T64);
    const int64_t ld = 2 * ld64;
    const int64_t nb = (D + kBoolBlock - 1) / kBoolBlock;
    const int nwd = (int)((D + 31) / 32);
    const int nrc = (int)((D + 63) / 64);
    // bulk update: the four-Russians tables where the grid of 512 x 512 tiles
    // fills the device, else the bit-sliced kernel
    const bool m4r = path == kBoolPathM4r || (path == kBoolPathAuto && D >= 8192);
    const int nwb = path == kBoolPathMfma ? kUpdateMfma : m4r ? 0 : bool_update_nwb(D);
    // the matrix-core update reads the round's pivot rows bit-transposed:
    // two buffers, round kb's in buffer kb % 2 (see below)
    uint32_t *const pt0 = static_cast<uint32_t *>(work);
    uint32_t *const pt1 =
        pt0 ? pt0 + bool_mfma_closure_work_bytes(D) / 2 / sizeof(uint32_t) : nullptr;
    hipError_t e = pivot_b(T, ld, D, 0, st);
    if (e != hipSuccess || nb == 1) return e;
    if ((e = panels_b(T, ld, D, 0, st)) != hipSuccess) return e;
    Aux *aux = (nb > 2 && !serial) ? aux_acquire(st, aux_create) : nullptr;
    for (int64_t kb = 0; kb < nb; kb++) {
        const BBlock b = bblock(D, kb);
        const double bs = b.bs;
        uint32_t *const pt = (kb & 1) ? pt1 : pt0;
        if (kb + 1 == nb || !aux) {
            if (aux && kb > 0) e = hipStreamWaitEvent(st, aux->ev_aux[(kb - 1) & 1], 0);
            const double rest = (double)D - bs;
            if (e == hipSuccess)
                e = update_b(T, ld, D, kb, BRect{0, nrc, b.rl, b.rh, 0, b.wl, b.wh, nwd}, nwb,
                             rest * rest * bs, st, false, pt);
            if (e == hipSuccess && kb + 1 < nb) e = pivot_b(T, ld, D, kb + 1, st);
            if (e == hipSuccess && kb + 1 < nb) e = panels_b(T, ld, D, kb + 1, st);
            if (e != hipSuccess) break;
            continue;
        }
        const BBlock n = bblock(D, kb + 1);
        const double bs1 = n.bs, rest2 = (double)D - bs - bs1;
        // the matrix-core update's transposed pivot rows of round kb on this
        // stream, right after panels(kb) (the chain is the shorter side), into
        // buffer kb % 2: B(kb - 1) may still read the other one, and round
        // kb + 2 rewrites this one only after A(kb + 1), which waits for B(kb)
        const bool pre = nwb == kUpdateMfma;
        if (pre) e = launch_bool_pivot_transpose(pt, T, ld, D, b.k0, b.bs, st);
        // B(kb) on the second stream, after panels(kb), behind B(kb-1)
        if (e == hipSuccess) e = hipEventRecord(aux->ev_main, st);
        if (e == hipSuccess) e = hipStreamWaitEvent(aux->stream, aux->ev_main, 0);
        if (e == hipSuccess)
            e = update_b(T, ld, D, kb, BRect{0, nrc, b.rl, n.rh, 0, b.wl, n.wh, nwd}, nwb,
                         rest2 * rest2 * bs, aux->stream, false, pt, pre);
        if (e == hipSuccess) e = hipEventRecord(aux->ev_aux[kb & 1], aux->stream);
        // A(kb) writes row block kb+1, which B(kb-1) writes too
        if (e == hipSuccess && kb > 0) e = hipStreamWaitEvent(st, aux->ev_aux[(kb - 1) & 1], 0);
        // A(kb): row block kb+1 (every word outside block kb), then column
        // block kb+1 (rows outside blocks kb and kb+1)
        if (e == hipSuccess)
            e = lookahead_b(T, ld, D, kb, BRect{n.rl, n.rh, n.rh, n.rh, 0, b.wl, b.wh, nwd},
                            BRect{0, nrc, b.rl, n.rh, n.wl, n.wh, n.wh, n.wh},
                            bs1 * ((double)D - bs) * bs + rest2 * bs1 * bs, st);
        if (e == hipSuccess) e = pivot_b(T, ld, D, kb + 1, st);
        if (e == hipSuccess) e = panels_b(T, ld, D, kb + 1, st);
        if (e != hipSuccess) break;
    }
    if (aux) aux_release(aux);
    return e;
}

}  // namespace sr
