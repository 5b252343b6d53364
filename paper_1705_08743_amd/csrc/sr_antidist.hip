// Anti-distance semiring product and blocked Floyd-Warshall closure on
// gfx950 (uint16 storage; uint8 data are widened by the caller).
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

#include <algorithm>

#include "sr_internal.h"
#include "sr_tiles.h"

namespace sr {
namespace {

using dev::tile_closure;
using dev::wave_tile;

constexpr int kPanelNW = 16;  // 32 columns per wave in the panel phase

// ---------------------------------------------------------------------------
template <int NW, bool S8>
__global__ void __launch_bounds__(256)
k_ad_mul(uint16_t *C, int64_t ldc, const uint16_t *A, int64_t lda, const uint16_t *B,
         int64_t ldb, int64_t R, int K, int64_t N, int accumulate) {
    constexpr int CW = 2 * NW;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform per wave
    const int64_t row0 = ((int64_t)blockIdx.y * 4 + wave) * 64;
    const int64_t col0 = (int64_t)blockIdx.x * CW;
    if (row0 >= R) return;
    const int nrows = (int)min<int64_t>(64, R - row0);
    const int ncols = (int)min<int64_t>(CW, N - col0);
    wave_tile<NW, S8>(C + row0 * ldc + col0, ldc, A + row0 * lda, lda, B + col0, ldb, nrows,
                      ncols, ldb - col0, K, accumulate != 0, false);
}

template <bool S8>
__global__ void __launch_bounds__(256) k_ad_fw_pivot(uint16_t *T, int64_t ld, int64_t k0, int bs) {
    __shared__ uint32_t lds_row[2 * 64];
    __shared__ uint32_t lds_col[2 * 128];
    tile_closure<S8>(T + k0 * ld + k0, ld, bs, lds_row, lds_col);
}

// Phase 2.  Workgroups [0, n_rowwg) take the row panel: two 64-row halves of
// the pivot rows times two 32-column chunks (the chunks outside the pivot
// block, two per workgroup).  The rest take the column panel: one 64-row chunk
// outside the pivot block times the four 32-column chunks of the pivot block.
// Every panel tile is read and written by one workgroup only, and a barrier
// separates its reads from its writes.
template <bool S8>
__global__ void __launch_bounds__(256)
k_ad_fw_panels(uint16_t *T, int64_t ld, int D, int k0, int bs, int n_rowwg) {
    constexpr int NW = kPanelNW, CW = 2 * NW;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform per wave
    if ((int)blockIdx.x < n_rowwg) {
        const int kc0 = k0 / CW, kc1 = (k0 + bs + CW - 1) / CW;
        const int cc = 2 * (int)blockIdx.x + (wave >> 1);
        const int c = cc < kc0 ? cc : cc + (kc1 - kc0);
        const int64_t col0 = (int64_t)c * CW;
        const int rofs = (wave & 1) * 64;
        const int nrows = min(64, bs - rofs);
        const int ncols = (int)min<int64_t>(CW, (int64_t)D - col0);
        const int64_t r0 = (int64_t)k0 + rofs;
        wave_tile<NW, S8>(T + r0 * ld + col0, ld, T + r0 * ld + k0, ld, T + (int64_t)k0 * ld + col0,
                          ld, nrows, ncols, ld - col0, bs, true, true);
    } else {
        const int kr0 = k0 / 64, kr1 = (k0 + bs + 63) / 64;
        const int rc = (int)blockIdx.x - n_rowwg;
        const int rchunk = rc < kr0 ? rc : rc + (kr1 - kr0);
        const int64_t row0 = (int64_t)rchunk * 64;
        const int nrows = (int)min<int64_t>(64, (int64_t)D - row0);
        const int cofs = wave * CW;
        const int ncols = min(CW, bs - cofs);
        wave_tile<NW, S8>(T + row0 * ld + k0 + cofs, ld, T + row0 * ld + k0, ld,
                          T + (int64_t)k0 * ld + k0 + cofs, ld, nrows, ncols, ld - k0 - cofs, bs,
                          true, true);
    }
}

// Phase 3.  Each wave owns a 64-row x 2NW-column tile outside the pivot rows
// and columns; the four waves of a workgroup share the column chunk, so they
// read the same pivot-row segments through the scalar cache.
template <int NW, bool S8>
__global__ void __launch_bounds__(256) k_ad_fw_update(uint16_t *T, int64_t ld, int D, int k0, int bs) {
    constexpr int CW = 2 * NW;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform per wave
    const int kc0 = k0 / CW, kc1 = (k0 + bs + CW - 1) / CW;
    const int cc = (int)blockIdx.x;
    const int c = cc < kc0 ? cc : cc + (kc1 - kc0);
    const int kr0 = k0 / 64, kr1 = (k0 + bs + 63) / 64;
    const int rc = (int)blockIdx.y * 4 + wave;
    const int rchunk = rc < kr0 ? rc : rc + (kr1 - kr0);
    const int64_t row0 = (int64_t)rchunk * 64, col0 = (int64_t)c * CW;
    if (row0 >= D) return;
    const int nrows = (int)min<int64_t>(64, (int64_t)D - row0);
    const int ncols = (int)min<int64_t>(CW, (int64_t)D - col0);
    wave_tile<NW, S8>(T + row0 * ld + col0, ld, T + row0 * ld + k0, ld, T + (int64_t)k0 * ld + col0,
                      ld, nrows, ncols, ld - col0, bs, true, false);
}

// uint8 <-> uint16, 8 entries per thread; rows padded with zeros up to the
// next multiple of 8 in the destination of a widening.
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
            v[i] = (uint16_t)((w.x >> (8 * i)) & 0xFFu);
            v[4 + i] = (uint16_t)((w.y >> (8 * i)) & 0xFFu);
        }
    } else {
#pragma unroll
        for (int i = 0; i < 8; i++) v[i] = (c0 + i < C) ? (uint16_t)s[i] : (uint16_t)0;
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
    uint8_t *d = dst + row * ldd + c0;
    if (c0 + 8 <= C) {
        uint2 o;
        o.x = (ww[0] & 0xFFu) | ((ww[0] >> 8) & 0xFF00u) | ((ww[1] & 0xFFu) << 16) |
              ((ww[1] >> 16) << 24);
        o.y = (ww[2] & 0xFFu) | ((ww[2] >> 8) & 0xFF00u) | ((ww[3] & 0xFFu) << 16) |
              ((ww[3] >> 16) << 24);
        *reinterpret_cast<uint2 *>(d) = o;
    } else {
        for (int i = 0; i < 8; i++)
            if (c0 + i < C) d[i] = (uint8_t)(ww[i >> 1] >> (16 * (i & 1)));
    }
}

// Column width of the wave tiles: wider tiles amortise the per-step work that
// is not a packed update; narrower ones give more waves for small products.
int pick_nw(int64_t R, int64_t N) {
    int nw = 32;
    while (nw > 8) {
        const int64_t waves = ((R + 63) / 64) * ((N + 2 * nw - 1) / (2 * nw));
        if (waves >= 4096) break;
        nw >>= 1;
    }
    return nw;
}

template <int NW, bool S8>
hipError_t mul_nw(uint16_t *C, int64_t ldc, const uint16_t *A, int64_t lda, const uint16_t *B,
                  int64_t ldb, int64_t R, int64_t K, int64_t N, bool acc, hipStream_t st) {
    const dim3 grid((unsigned)((N + 2 * NW - 1) / (2 * NW)), (unsigned)((R + 255) / 256));
    hipLaunchKernelGGL((k_ad_mul<NW, S8>), grid, dim3(256), 0, st, C, ldc, A, lda, B, ldb, R,
                       (int)K, N, acc ? 1 : 0);
    return hipGetLastError();
}

template <bool S8>
hipError_t mul_s(uint16_t *C, int64_t ldc, const uint16_t *A, int64_t lda, const uint16_t *B,
                 int64_t ldb, int64_t R, int64_t K, int64_t N, bool acc, hipStream_t st) {
    switch (pick_nw(R, N)) {
        case 32: return mul_nw<32, S8>(C, ldc, A, lda, B, ldb, R, K, N, acc, st);
        case 16: return mul_nw<16, S8>(C, ldc, A, lda, B, ldb, R, K, N, acc, st);
        default: return mul_nw<8, S8>(C, ldc, A, lda, B, ldb, R, K, N, acc, st);
    }
}

struct Round {
    int k0, bs;
    int n_rowwg, n_colwg;        // phase 2 grid
    int upd_x, upd_y;            // phase 3 grid
};

Round plan_round(int64_t D, int64_t kb, int nw) {
    Round r;
    r.k0 = (int)(kb * kAdBlock);
    r.bs = (int)std::min<int64_t>(kAdBlock, D - r.k0);
    const int pcw = 2 * kPanelNW;
    const int64_t nchunk_p = (D + pcw - 1) / pcw;
    const int kpc = (r.k0 + r.bs + pcw - 1) / pcw - r.k0 / pcw;
    r.n_rowwg = (int)((nchunk_p - kpc + 1) / 2);
    const int64_t nrch = (D + 63) / 64;
    const int kr = (r.k0 + r.bs + 63) / 64 - r.k0 / 64;
    r.n_colwg = (int)(nrch - kr);
    const int cw = 2 * nw;
    const int64_t nchunk_u = (D + cw - 1) / cw;
    const int kuc = (r.k0 + r.bs + cw - 1) / cw - r.k0 / cw;
    r.upd_x = (int)(nchunk_u - kuc);
    r.upd_y = (int)((nrch - kr + 3) / 4);
    return r;
}

int closure_nw(int64_t D) { return D >= 2048 ? 32 : (D >= 512 ? 16 : 8); }

template <bool S8>
hipError_t pivot_s(uint16_t *T, int64_t ld, const Round &r, hipStream_t st) {
    hipLaunchKernelGGL((k_ad_fw_pivot<S8>), dim3(1), dim3(256), 0, st, T, ld, (int64_t)r.k0, r.bs);
    return hipGetLastError();
}

template <bool S8>
hipError_t panels_s(uint16_t *T, int64_t ld, int64_t D, const Round &r, hipStream_t st) {
    const int n = r.n_rowwg + r.n_colwg;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_ad_fw_panels<S8>), dim3(n), dim3(256), 0, st, T, ld, (int)D, r.k0, r.bs,
                       r.n_rowwg);
    return hipGetLastError();
}

template <int NW, bool S8>
hipError_t update_nw(uint16_t *T, int64_t ld, int64_t D, const Round &r, hipStream_t st) {
    if (r.upd_x <= 0 || r.upd_y <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_ad_fw_update<NW, S8>), dim3(r.upd_x, r.upd_y), dim3(256), 0, st, T, ld,
                       (int)D, r.k0, r.bs);
    return hipGetLastError();
}

template <bool S8>
hipError_t update_s(uint16_t *T, int64_t ld, int64_t D, int nw, const Round &r, hipStream_t st) {
    switch (nw) {
        case 32: return update_nw<32, S8>(T, ld, D, r, st);
        case 16: return update_nw<16, S8>(T, ld, D, r, st);
        default: return update_nw<8, S8>(T, ld, D, r, st);
    }
}

template <bool S8>
hipError_t closure_s(uint16_t *T, int64_t ld, int64_t D, hipStream_t st) {
    const int nw = closure_nw(D);
    const int64_t nb = (D + kAdBlock - 1) / kAdBlock;
    for (int64_t kb = 0; kb < nb; kb++) {
        const Round r = plan_round(D, kb, nw);
        hipError_t e = pivot_s<S8>(T, ld, r, st);
        if (e != hipSuccess) return e;
        if (nb == 1) break;
        if ((e = panels_s<S8>(T, ld, D, r, st)) != hipSuccess) return e;
        if ((e = update_s<S8>(T, ld, D, nw, r, st)) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

hipError_t launch_ad_mul(bool s8, uint16_t *C, int64_t ldc, const uint16_t *A, int64_t lda,
                         const uint16_t *B, int64_t ldb, int64_t R, int64_t K, int64_t N,
                         bool accumulate, hipStream_t stream) {
    return s8 ? mul_s<true>(C, ldc, A, lda, B, ldb, R, K, N, accumulate, stream)
              : mul_s<false>(C, ldc, A, lda, B, ldb, R, K, N, accumulate, stream);
}

hipError_t launch_ad_closure(bool s8, uint16_t *T, int64_t ld, int64_t D, hipStream_t stream) {
    return s8 ? closure_s<true>(T, ld, D, stream) : closure_s<false>(T, ld, D, stream);
}

hipError_t launch_ad_fw_pivot(bool s8, uint16_t *T, int64_t ld, int64_t D, int64_t kb,
                              hipStream_t stream) {
    const Round r = plan_round(D, kb, closure_nw(D));
    return s8 ? pivot_s<true>(T, ld, r, stream) : pivot_s<false>(T, ld, r, stream);
}

hipError_t launch_ad_fw_panels(bool s8, uint16_t *T, int64_t ld, int64_t D, int64_t kb,
                               hipStream_t stream) {
    const Round r = plan_round(D, kb, closure_nw(D));
    return s8 ? panels_s<true>(T, ld, D, r, stream) : panels_s<false>(T, ld, D, r, stream);
}

hipError_t launch_ad_fw_update(bool s8, uint16_t *T, int64_t ld, int64_t D, int64_t kb,
                               hipStream_t stream) {
    const int nw = closure_nw(D);
    const Round r = plan_round(D, kb, nw);
    return s8 ? update_s<true>(T, ld, D, nw, r, stream) : update_s<false>(T, ld, D, nw, r, stream);
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
