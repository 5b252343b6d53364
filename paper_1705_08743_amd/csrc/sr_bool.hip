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
template <int NWB, bool FULL>
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
#pragma unroll
                for (int u = 0; u < KU; u++) {
                    const uint32_t m = (uint32_t)__builtin_amdgcn_sbfe(a, g + u, 1);
                    const kconst uint32_t *brow = (const kconst uint32_t *)(b0 + u * ldb);
#pragma unroll
                    for (int w = 0; w < NWB; w++)
                        acc[w] = __builtin_amdgcn_bitop3_b32(brow[w], m, acc[w], 0xEA);
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
template <int NWB>
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
            bool_tile_body<NWB, true>(C, ldc, A, lda, B, ldb, nrows, NWB, K, accumulate,
                                      sync_before_store);
        else
            bool_tile_body<NWB, false>(C, ldc, A, lda, B, ldb, nrows, nw, K, accumulate,
                                       sync_before_store);
        return;
    }
    for (int c = 0; c < nw; c += 4) {
        const int n = min(4, nw - c);
        if (n == 4)
            bool_tile_body<4, true>(C + c, ldc, A, lda, B + c, ldb, nrows, 4, K, accumulate, false);
        else
            bool_tile_body<4, false>(C + c, ldc, A, lda, B + c, ldb, nrows, n, K, accumulate, false);
    }
    if (sync_before_store) __syncthreads();
}

template <int NWB>
__global__ void __launch_bounds__(256)
k_bool_mul(uint32_t *C, int64_t ldc, const uint32_t *A, int64_t lda, const uint32_t *B, int64_t ldb,
           int64_t R, int K, int64_t nwords, int accumulate) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform per wave
    const int64_t row0 = ((int64_t)blockIdx.y * 4 + wave) * 64;
    const int64_t w0 = (int64_t)blockIdx.x * NWB;
    if (row0 >= R) return;
    bool_tile<NWB>(C + row0 * ldc + w0, ldc, A + row0 * lda, lda, B + w0, ldb,
                   (int)min<int64_t>(64, R - row0), (int)min<int64_t>(NWB, nwords - w0), ldb - w0,
                   K, accumulate != 0, false);
}

// Pivot tile closure: 256 threads, thread t holds row t of the tile as 8
// words (256 bits).  Step k: the owner of row k publishes it in LDS (two
// alternating buffers, one barrier per step); every row with bit k set ORs it
// in.  Row k does not change during step k.  nwv: valid words of a tile row.
__global__ void __launch_bounds__(256)
k_bool_fw_pivot(uint32_t *T, int64_t ld, int64_t k0, int bs, int nwv) {
    __shared__ uint32_t buf[2 * 8];
    uint32_t *tile = T + k0 * ld + (k0 >> 5);
    const int t = threadIdx.x;
    const bool live = t < bs;
    uint32_t r[8];
#pragma unroll
    for (int j = 0; j < 8; j++) r[j] = (live && j < nwv) ? tile[(int64_t)t * ld + j] : 0u;
#pragma unroll
    for (int w = 0; w < 8; w++) {
        const int kb = 32 * w;
        if (kb >= bs) break;
        const int kn = min(32, bs - kb);
        for (int b = 0; b < kn; b++) {
            uint32_t *pb = buf + (b & 1) * 8;
            if (t == kb + b) {
                reinterpret_cast<uint4 *>(pb)[0] = uint4{r[0], r[1], r[2], r[3]};
                reinterpret_cast<uint4 *>(pb)[1] = uint4{r[4], r[5], r[6], r[7]};
            }
            __syncthreads();
            const uint4 p0 = reinterpret_cast<const uint4 *>(pb)[0];
            const uint4 p1 = reinterpret_cast<const uint4 *>(pb)[1];
            const uint32_t m = (uint32_t)__builtin_amdgcn_sbfe(r[w], b, 1);
            r[0] |= p0.x & m;
            r[1] |= p0.y & m;
            r[2] |= p0.z & m;
            r[3] |= p0.w & m;
            r[4] |= p1.x & m;
            r[5] |= p1.y & m;
            r[6] |= p1.z & m;
            r[7] |= p1.w & m;
        }
    }
    if (live)
#pragma unroll
        for (int j = 0; j < 8; j++)
            if (j < nwv) tile[(int64_t)t * ld + j] = r[j];
}

// Phase 2.  Workgroups [0, n_rowwg): the 256 pivot rows (4 waves x 64) times
// one 8-word (256-column) chunk outside the pivot block; reads of the chunk
// precede its writes (barrier).  The rest: column panel, each wave 64 rows
// outside the pivot block times the 8 pivot words; a lane reads and writes
// only its own row.
__global__ void __launch_bounds__(256)
k_bool_fw_panels(uint32_t *T, int64_t ld, int D, int k0, int bs, int n_rowwg) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform per wave
    const int64_t nwd = ((int64_t)D + 31) >> 5;
    const int kw0 = k0 >> 5;
    const int kpw = (int)min<int64_t>(8, nwd - kw0);
    if ((int)blockIdx.x < n_rowwg) {
        const int cc = (int)blockIdx.x;
        const int64_t c = cc < (kw0 >> 3) ? cc : cc + 1;
        const int64_t w0 = c * 8;
        const int rofs = wave * 64;
        const int64_t r0 = (int64_t)k0 + rofs;
        bool_tile<8>(T + r0 * ld + w0, ld, T + r0 * ld + kw0, ld, T + (int64_t)k0 * ld + w0, ld,
                     min(64, bs - rofs), (int)min<int64_t>(8, nwd - w0), ld - w0, bs, true, true);
    } else {
        const int kr0 = k0 / 64, kr1 = (k0 + bs + 63) / 64;
        const int rc = ((int)blockIdx.x - n_rowwg) * 4 + wave;
        const int rchunk = rc < kr0 ? rc : rc + (kr1 - kr0);
        const int64_t row0 = (int64_t)rchunk * 64;
        if (row0 >= D) return;
        bool_tile<8>(T + row0 * ld + kw0, ld, T + row0 * ld + kw0, ld,
                     T + (int64_t)k0 * ld + kw0, ld, (int)min<int64_t>(64, (int64_t)D - row0), kpw,
                     ld - kw0, bs, true, false);
    }
}

// Phase 3.  Rows outside the pivot block, all column words in chunks of NWB.
// A chunk may contain pivot columns: there the update recomputes
// T_iK (|)= T_iK * T_KK, which phase 2 already applied and which cannot
// change T_iK again (T_KK is closed), so the same bits are written back.
template <int NWB>
__global__ void __launch_bounds__(256) k_bool_fw_update(uint32_t *T, int64_t ld, int D, int k0, int bs) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform per wave
    const int64_t nwd = ((int64_t)D + 31) >> 5;
    const int kr0 = k0 / 64, kr1 = (k0 + bs + 63) / 64;
    const int rc = (int)blockIdx.y * 4 + wave;
    const int rchunk = rc < kr0 ? rc : rc + (kr1 - kr0);
    const int64_t row0 = (int64_t)rchunk * 64, w0 = (int64_t)blockIdx.x * NWB;
    if (row0 >= D) return;
    bool_tile<NWB>(T + row0 * ld + w0, ld, T + row0 * ld + (k0 >> 5), ld, T + (int64_t)k0 * ld + w0,
                   ld, (int)min<int64_t>(64, (int64_t)D - row0), (int)min<int64_t>(NWB, nwd - w0),
                   ld - w0, bs, true, false);
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
hipError_t update_nwb(uint32_t *T, int64_t ld, int64_t D, int k0, int bs, hipStream_t st) {
    const int64_t nwd = (D + 31) / 32;
    const int64_t nrch = (D + 63) / 64;
    const int kr = (k0 + bs + 63) / 64 - k0 / 64;
    const dim3 grid((unsigned)((nwd + NWB - 1) / NWB), (unsigned)((nrch - kr + 3) / 4));
    if (grid.x == 0 || grid.y == 0) return hipSuccess;
    hipLaunchKernelGGL((k_bool_fw_update<NWB>), grid, dim3(256), 0, st, T, ld, (int)D, k0, bs);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_bool_mul(uint64_t *C, int64_t ldc, const uint64_t *A, int64_t lda,
                           const uint64_t *B, int64_t ldb, int64_t R, int64_t K, int64_t N,
                           bool accumulate, hipStream_t stream) {
    uint32_t *c = reinterpret_cast<uint32_t *>(C);
    const uint32_t *a = reinterpret_cast<const uint32_t *>(A);
    const uint32_t *b = reinterpret_cast<const uint32_t *>(B);
    const int64_t nwords = (N + 31) / 32;
    int nwb = 32;
    while (nwb > 8 && ((R + 63) / 64) * ((nwords + nwb - 1) / nwb) < 4096) nwb >>= 1;
    switch (nwb) {
        case 32: return mul_nwb<32>(c, 2 * ldc, a, 2 * lda, b, 2 * ldb, R, K, nwords, accumulate, stream);
        case 16: return mul_nwb<16>(c, 2 * ldc, a, 2 * lda, b, 2 * ldb, R, K, nwords, accumulate, stream);
        default: return mul_nwb<8>(c, 2 * ldc, a, 2 * lda, b, 2 * ldb, R, K, nwords, accumulate, stream);
    }
}

hipError_t launch_bool_closure(uint64_t *T64, int64_t ld64, int64_t D, bool serial,
                               hipStream_t st) {
    (void)serial;
    uint32_t *T = reinterpret_cast<uint32_t *>(T64);
    const int64_t ld = 2 * ld64;
    const int64_t nb = (D + kBoolBlock - 1) / kBoolBlock;
    const int64_t nwd = (D + 31) / 32;
    const int64_t nrch = (D + 63) / 64;
    const int nwb = D >= 8192 ? 32 : (D >= 2048 ? 16 : 8);
    for (int64_t kb = 0; kb < nb; kb++) {
        const int k0 = (int)(kb * kBoolBlock);
        const int bs = (int)std::min<int64_t>(kBoolBlock, D - k0);
        const int nwv = (int)std::min<int64_t>(8, nwd - k0 / 32);
        const bool prof = prof_on();
        const double dbs = bs, rest = (double)(D - bs);
        if (prof) prof_begin(st);
        hipLaunchKernelGGL(k_bool_fw_pivot, dim3(1), dim3(256), 0, st, T, ld, (int64_t)k0, bs, nwv);
        hipError_t e = hipGetLastError();
        if (prof) prof_end(st, 0, 0, dbs * dbs * dbs);
        if (e != hipSuccess) return e;
        if (nb == 1) break;
        const int64_t nchunks = (nwd + 7) / 8;
        const int n_rowwg = (int)(nchunks - 1);
        const int kr = (k0 + bs + 63) / 64 - k0 / 64;
        const int n_colwg = (int)((nrch - kr + 3) / 4);
        if (prof) prof_begin(st);
        hipLaunchKernelGGL(k_bool_fw_panels, dim3(n_rowwg + n_colwg), dim3(256), 0, st, T, ld,
                           (int)D, k0, bs, n_rowwg);
        e = hipGetLastError();
        if (prof) prof_end(st, 0, 1, 2.0 * rest * dbs * dbs);
        if (e != hipSuccess) return e;
        if (prof) prof_begin(st);
        switch (nwb) {
            case 32: e = update_nwb<32>(T, ld, D, k0, bs, st); break;
            case 16: e = update_nwb<16>(T, ld, D, k0, bs, st); break;
            default: e = update_nwb<8>(T, ld, D, k0, bs, st); break;
        }
        if (prof) prof_end(st, 0, 2, rest * rest * dbs);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace sr
