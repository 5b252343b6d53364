// The two ends of the closure by repeated squaring (eq. trcl) for entries of
// 16 bits (uint16, or the binary16 form of uint8 data) and 32 bits.
//
// prep:   P := I (+) T (the diagonal becomes the multiplicative one S), and
//         the squarings' change flags are cleared -- one launch in place of a
//         copy, a diagonal write and a fill.
// finish: with P = (I (+) A)^m, m >= D - 1, the closure A * P needs no
//         product.  Off the diagonal (A * P)_ij is a best path of 1 .. m + 1
//         edges and P_ij one of 1 .. m edges (the I term is the additive zero
//         there); a best path never needs more than D - 1 <= m edges, because
//         dropping a cycle never lowers its value (x (*) y <= y), so the two
//         agree.  On the diagonal (A * P)_ii is the best cycle through i:
//         the first edge i -> j, then a best path j -> i (P_ii = S covers the
//         self loop).  So T := P with T_ii := (+)_j A_ij (*) P_ji, an O(D^2)
//         pass in place of the last O(D^3) product.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "sr_internal.h"

namespace sr {
namespace {

// a (*) b = max(a + b - S, 0) on one entry; S8: binary16 bit patterns of the
// integers 0 .. 255 (S = 255), exact in binary16 and in float.
template <int ES, bool S8>
__device__ __forceinline__ uint32_t otimes(uint32_t a, uint32_t b) {
    if (ES == 4) {
        const uint64_t s = (uint64_t)a + b;
        return s > 0xFFFFFFFFull ? (uint32_t)(s - 0xFFFFFFFFull) : 0u;
    }
    if (S8) {
        const float x = (float)__builtin_bit_cast(_Float16, (uint16_t)a);
        const float y = (float)__builtin_bit_cast(_Float16, (uint16_t)b);
        const float r = fmaxf(x + y - 255.0f, 0.0f);
        return __builtin_bit_cast(uint16_t, (_Float16)r);
    }
    const uint32_t s = a + b;
    return s > 0xFFFFu ? s - 0xFFFFu : 0u;
}

template <int ES>
__device__ __forceinline__ uint32_t load_entry(const uint8_t *p) {
    return ES == 4 ? *reinterpret_cast<const uint32_t *>(p) : *reinterpret_cast<const uint16_t *>(p);
}

template <int ES>
__device__ __forceinline__ void store_entry(uint8_t *p, uint32_t v) {
    if (ES == 4)
        *reinterpret_cast<uint32_t *>(p) = v;
    else
        *reinterpret_cast<uint16_t *>(p) = (uint16_t)v;
}

// Copies row r of src into dst (the first D entries, in 16-byte groups; a
// group that ends past entry D is copied entry by entry), with entry `diag`
// of the row replaced by `dv`.  Rows start 16-byte aligned.
template <int ES>
__device__ __forceinline__ void copy_group(uint8_t *dst, const uint8_t *src, int64_t g, int64_t D,
                                           int64_t diag, uint32_t dv) {
    constexpr int E = 16 / ES;
    const int64_t c0 = g * E;
    if (c0 + E <= D) {
        uint4 v = *reinterpret_cast<const uint4 *>(src + c0 * ES);
        if (diag >= c0 && diag < c0 + E) {
            uint32_t w[4] = {v.x, v.y, v.z, v.w};
            const int o = (int)(diag - c0);
            if (ES == 4)
                w[o] = dv;
            else
                w[o >> 1] = (o & 1) ? ((w[o >> 1] & 0xFFFFu) | (dv << 16))
                                    : ((w[o >> 1] & 0xFFFF0000u) | (dv & 0xFFFFu));
            v = make_uint4(w[0], w[1], w[2], w[3]);
        }
        *reinterpret_cast<uint4 *>(dst + c0 * ES) = v;
    } else {
        for (int64_t c = c0; c < D; c++)
            store_entry<ES>(dst + c * ES, c == diag ? dv : load_entry<ES>(src + c * ES));
    }
}

// P := I (+) T over the D x D matrix (strides in bytes, multiples of 16);
// flags[0 .. nflags) := 0.  Grid-stride over 16-byte groups.
template <int ES>
__global__ void __launch_bounds__(256)
k_power_prep(uint8_t *P, int64_t ldp, const uint8_t *T, int64_t ldt, int64_t D, uint32_t one,
             int *flags, int nflags) {
    if (blockIdx.x == 0 && (int)threadIdx.x < nflags) flags[threadIdx.x] = 0;
    constexpr int E = 16 / ES;
    const int64_t gpr = (D + E - 1) / E, total = D * gpr;
    for (int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x; g < total;
         g += (int64_t)gridDim.x * 256) {
        const int64_t r = g / gpr;
        copy_group<ES>(P + r * ldp, T + r * ldt, g % gpr, D, r, one);
    }
}

// T := P with T_ii := (+)_j T_ij (*) P_ji, read before T is written.  One
// wave per row i (four rows per workgroup): lane l takes j = l, l + 64, ...
// (row i of T read contiguously, column i of P one entry per row j, from L2),
// the wave's maximum is d_i; after a barrier the wave copies row i of P into
// T with d_i on the diagonal.  Only this wave reads or writes row i of T.
template <int ES, bool S8>
__global__ void __launch_bounds__(256)
k_power_finish(uint8_t *T, int64_t ldt, const uint8_t *P, int64_t ldp, int64_t D) {
    constexpr int E = 16 / ES, U = 4;
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    uint32_t acc = 0;
    if (i < D) {
        const uint8_t *trow = T + i * ldt;
        const uint8_t *pcol = P + i * ES;
        for (int64_t j0 = lane; j0 < D; j0 += 64 * U) {
            uint32_t a[U], b[U];
#pragma unroll
            for (int u = 0; u < U; u++) {
                const int64_t j = j0 + 64 * u;
                a[u] = j < D ? load_entry<ES>(trow + j * ES) : 0u;
                b[u] = j < D ? load_entry<ES>(pcol + j * ldp) : 0u;
            }
#pragma unroll
            for (int u = 0; u < U; u++) acc = max(acc, otimes<ES, S8>(a[u], b[u]));
        }
        // (non-negative binary16 values order like their bit patterns)
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) acc = max(acc, (uint32_t)__shfl_xor((int)acc, o, 64));
    }
    __syncthreads();
    if (i >= D) return;
    const int64_t gpr = (D + E - 1) / E;
    for (int64_t g = lane; g < gpr; g += 64)
        copy_group<ES>(T + i * ldt, P + i * ldp, g, D, i, acc);
}

}  // namespace

hipError_t launch_power_prep(int es, void *P, int64_t ldp, const void *T, int64_t ldt, int64_t D,
                             uint32_t one, int *flags, int nflags, hipStream_t st) {
    if (D <= 0) return hipSuccess;
    const int64_t groups = D * ((D * es + 15) / 16);
    const unsigned blocks = (unsigned)std::min<int64_t>((groups + 255) / 256, 2048);
    uint8_t *p = static_cast<uint8_t *>(P);
    const uint8_t *t = static_cast<const uint8_t *>(T);
    if (es == 4)
        hipLaunchKernelGGL(k_power_prep<4>, dim3(blocks), dim3(256), 0, st, p, ldp * 4, t, ldt * 4,
                           D, one, flags, nflags);
    else
        hipLaunchKernelGGL(k_power_prep<2>, dim3(blocks), dim3(256), 0, st, p, ldp * 2, t, ldt * 2,
                           D, one, flags, nflags);
    return hipGetLastError();
}

hipError_t launch_power_finish(int es, bool s8, void *T, int64_t ldt, const void *P, int64_t ldp,
                               int64_t D, hipStream_t st) {
    if (D <= 0) return hipSuccess;
    const dim3 grid((unsigned)((D + 3) / 4));
    uint8_t *t = static_cast<uint8_t *>(T);
    const uint8_t *p = static_cast<const uint8_t *>(P);
    if (es == 4)
        hipLaunchKernelGGL((k_power_finish<4, false>), grid, dim3(256), 0, st, t, ldt * 4, p,
                           ldp * 4, D);
    else if (s8)
        hipLaunchKernelGGL((k_power_finish<2, true>), grid, dim3(256), 0, st, t, ldt * 2, p,
                           ldp * 2, D);
    else
        hipLaunchKernelGGL((k_power_finish<2, false>), grid, dim3(256), 0, st, t, ldt * 2, p,
                           ldp * 2, D);
    return hipGetLastError();
}

}  // namespace sr
