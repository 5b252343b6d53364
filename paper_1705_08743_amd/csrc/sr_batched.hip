// Batched anti-distance closure: many independent graphs of uneven size in
// one launch.  Workgroup g closes graph g of a descriptor array that the host
// has sorted largest-first, so the hardware dispatcher hands out the longest
// jobs first and fills the machine with the short ones as it drains
// (longest-processing-time-first list scheduling).
//
// Per graph (256 threads):
//   D <= kAdBlock: the whole matrix is one tile closed in registers + LDS
//                  (the pivot routine of the blocked closure).
//   D >  kAdBlock: the blocked Floyd-Warshall of sr_antidist.hip inside the
//                  workgroup: per round the pivot tile, then the panel tiles,
//                  then the remaining tiles, each phase shared by the four
//                  waves and separated by workgroup barriers.
//
// Inside one phase, waves update panel tiles that other waves read (a row of
// the pivot rows is both an output and an operand).  This is exact: with
// T_KK closed, T_Kj (+) T_KK * Y gives the same value for every Y between the
// old and the new T_Kj, and the same holds for T_iK (+) Y * T_KK; in phase 3
// the row panel may likewise be read old or new.  Entries are never torn
// (16-bit entries written by 32/128-bit stores).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sr_internal.h"
#include "sr_tiles.h"

namespace sr {
namespace {

using dev::tile_closure;
using dev::wave_tile;

constexpr int kBNW = 16;  // 32-column wave tiles
constexpr int kBCW = 2 * kBNW;

template <bool S8>
__device__ void blocked_closure_wg(uint16_t *T, int64_t ld, int D, uint32_t *lds_row,
                                   uint32_t *lds_col) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform per wave
    const int nb = (D + kAdBlock - 1) / kAdBlock;
    const int nrch = (D + 63) / 64;
    const int ncch = (D + kBCW - 1) / kBCW;
    for (int kb = 0; kb < nb; kb++) {
        const int k0 = kb * kAdBlock;
        const int bs = min(kAdBlock, D - k0);
        tile_closure<S8>(T + (int64_t)k0 * ld + k0, ld, bs, lds_row, lds_col);
        if (nb == 1) break;
        __syncthreads();
        const int kr0 = k0 / 64, kr = (k0 + bs + 63) / 64 - kr0;
        const int kc0 = k0 / kBCW, kc = (k0 + bs + kBCW - 1) / kBCW - kc0;
        const int nrx = nrch - kr, ncx = ncch - kc;
        // phase 2: row-panel items (pivot-row half h, column chunk c), then
        // column-panel items (row chunk r, pivot column chunk q)
        const int n_row_items = 2 * ncx, n_items2 = n_row_items + 4 * nrx;
        for (int it = wave; it < n_items2; it += 4) {
            if (it < n_row_items) {
                const int h = it & 1, cc = it >> 1;
                const int c = cc < kc0 ? cc : cc + kc;
                const int64_t col0 = (int64_t)c * kBCW, r0 = (int64_t)k0 + 64 * h;
                wave_tile<1, kBNW, S8>(T + r0 * ld + col0, ld, T + r0 * ld + k0, ld,
                                    T + (int64_t)k0 * ld + col0, ld, min(64, bs - 64 * h),
                                    (int)min<int64_t>(kBCW, D - col0), ld - col0, bs, true, false);
            } else {
                const int j = it - n_row_items;
                const int rr = j >> 2, q = j & 3;
                const int rch = rr < kr0 ? rr : rr + kr;
                const int64_t row0 = (int64_t)rch * 64;
                wave_tile<1, kBNW, S8>(T + row0 * ld + k0 + q * kBCW, ld, T + row0 * ld + k0, ld,
                                    T + (int64_t)k0 * ld + k0 + q * kBCW, ld,
                                    (int)min<int64_t>(64, D - row0), min(kBCW, bs - q * kBCW),
                                    ld - k0 - q * kBCW, bs, true, false);
            }
        }
        __syncthreads();
        // phase 3: every (row chunk, column chunk) outside the pivot block
        const int n_items3 = nrx * ncx;
        for (int it = wave; it < n_items3; it += 4) {
            const int rr = it / ncx, cc = it % ncx;
            const int rch = rr < kr0 ? rr : rr + kr;
            const int c = cc < kc0 ? cc : cc + kc;
            const int64_t row0 = (int64_t)rch * 64, col0 = (int64_t)c * kBCW;
            wave_tile<1, kBNW, S8>(T + row0 * ld + col0, ld, T + row0 * ld + k0, ld,
                                T + (int64_t)k0 * ld + col0, ld, (int)min<int64_t>(64, D - row0),
                                (int)min<int64_t>(kBCW, D - col0), ld - col0, bs, true, false);
        }
        __syncthreads();
    }
}

template <bool S8>
__global__ void __launch_bounds__(256) k_ad_batched(const BatchDesc *desc) {
    __shared__ uint32_t lds_row[2 * 64];
    __shared__ uint32_t lds_col[2 * 128];
    const BatchDesc d = desc[blockIdx.x];
    if (d.D <= 0) return;
    if (d.D <= kAdBlock)
        tile_closure<S8>(d.T, d.ld, d.D, lds_row, lds_col);
    else
        blocked_closure_wg<S8>(d.T, d.ld, d.D, lds_row, lds_col);
}

// uint8 <-> uint16 for every graph of a batch (workgroup g: graph g).
__global__ void __launch_bounds__(256) k_batch_widen(const BatchDesc *desc) {
    const BatchDesc d = desc[blockIdx.x];
    const int64_t gpr = ((int64_t)d.D + 7) >> 3;
    for (int64_t g = threadIdx.x; g < (int64_t)d.D * gpr; g += 256) {
        const int64_t row = g / gpr, c0 = (g % gpr) * 8;
        const uint8_t *s = d.T8 + row * d.ld8 + c0;
        uint16_t v[8];
#pragma unroll
        for (int i = 0; i < 8; i++) v[i] = (c0 + i < d.D) ? (uint16_t)s[i] : (uint16_t)0;
        uint4 o;
        o.x = v[0] | ((uint32_t)v[1] << 16);
        o.y = v[2] | ((uint32_t)v[3] << 16);
        o.z = v[4] | ((uint32_t)v[5] << 16);
        o.w = v[6] | ((uint32_t)v[7] << 16);
        *reinterpret_cast<uint4 *>(d.T + row * d.ld + c0) = o;
    }
}

__global__ void __launch_bounds__(256) k_batch_narrow(const BatchDesc *desc) {
    const BatchDesc d = desc[blockIdx.x];
    const int64_t gpr = ((int64_t)d.D + 7) >> 3;
    for (int64_t g = threadIdx.x; g < (int64_t)d.D * gpr; g += 256) {
        const int64_t row = g / gpr, c0 = (g % gpr) * 8;
        const uint4 w = *reinterpret_cast<const uint4 *>(d.T + row * d.ld + c0);
        const uint32_t ww[4] = {w.x, w.y, w.z, w.w};
        uint8_t *dst = d.T8 + row * d.ld8 + c0;
#pragma unroll
        for (int i = 0; i < 8; i++)
            if (c0 + i < d.D) dst[i] = (uint8_t)(ww[i >> 1] >> (16 * (i & 1)));
    }
}

}  // namespace

hipError_t launch_ad_closure_batched(bool s8, const BatchDesc *desc, int64_t count, int32_t max_d,
                                     hipStream_t stream) {
    (void)max_d;
    if (count <= 0) return hipSuccess;
    const dim3 grid((unsigned)count);
    if (s8) {
        hipLaunchKernelGGL(k_batch_widen, grid, dim3(256), 0, stream, desc);
        hipLaunchKernelGGL(k_ad_batched<true>, grid, dim3(256), 0, stream, desc);
        hipLaunchKernelGGL(k_batch_narrow, grid, dim3(256), 0, stream, desc);
    } else {
        hipLaunchKernelGGL(k_ad_batched<false>, grid, dim3(256), 0, stream, desc);
    }
    return hipGetLastError();
}

}  // namespace sr
