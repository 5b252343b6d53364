// Device-side building blocks shared by the anti-distance kernels
// (sr_antidist.hip) and the batched closure (sr_batched.hip).
//
// Storage: anti-distance entries in 16-bit words, in one of two forms.
//   S = 65535 (uint16 data): the entries themselves;
//     a (x) b = max(a + b - S, 0) = b -sat (S - a), the paper's rewriting of
//     a + b - S as b - (S - a), done as one packed saturating subtract per
//     two entries (S - a is the complement), and (+) = max one packed max.
//   S = 255 (uint8 data, template flag S8): the entries' values as binary16
//     floats (0..255 are exact, as is every sum and difference below);
//     a (x) b (+) acc = max(acc, b + (a - 255)): a result below zero can only
//     lose to acc >= 0, so no clamp is needed, and the products of two inner
//     steps enter the accumulator through one v_pk_maximum3_f16 -- three
//     packed operations per four updates instead of four.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sr {
namespace dev {

typedef uint16_t u16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 h16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ u16x2 as_pair(uint32_t x) { return __builtin_bit_cast(u16x2, x); }
__device__ __forceinline__ uint32_t as_word(u16x2 x) { return __builtin_bit_cast(uint32_t, x); }
__device__ __forceinline__ h16x2 as_h(u16x2 x) { return __builtin_bit_cast(h16x2, x); }
__device__ __forceinline__ u16x2 as_u(h16x2 x) { return __builtin_bit_cast(u16x2, x); }

// uint8 value <-> its 16-bit working form (binary16 of the value).
__device__ __forceinline__ uint16_t u8_to_work(uint32_t v) {
    return __builtin_bit_cast(uint16_t, (_Float16)(float)v);
}
__device__ __forceinline__ uint8_t work_to_u8(uint16_t w) {
    return (uint8_t)(uint32_t)(float)__builtin_bit_cast(_Float16, w);
}

// Four uint8 values (one word, low byte first) -> their working forms as two
// packed pairs.  Each byte b is placed under the high byte 0x64, the binary16
// pattern of 1024 + b, and 1024 is subtracted in binary16: exact, with 0
// giving +0, the same bits as u8_to_work.
__device__ __forceinline__ void widen4(uint32_t w, uint32_t &lo, uint32_t &hi) {
    const h16x2 k = {(_Float16)1024.0f, (_Float16)1024.0f};
    lo = __builtin_bit_cast(uint32_t,
                            __builtin_bit_cast(h16x2, __builtin_amdgcn_perm(0x64646464u, w, 0x04010400u)) - k);
    hi = __builtin_bit_cast(uint32_t,
                            __builtin_bit_cast(h16x2, __builtin_amdgcn_perm(0x64646464u, w, 0x04030402u)) - k);
}
// The way back for two pairs holding working forms of 0..255: + 1024 puts
// each value in the low byte of its half, and one byte permute gathers them.
__device__ __forceinline__ uint32_t narrow4(uint32_t lo, uint32_t hi) {
    const h16x2 k = {(_Float16)1024.0f, (_Float16)1024.0f};
    const uint32_t a = __builtin_bit_cast(uint32_t, __builtin_bit_cast(h16x2, lo) + k);
    const uint32_t b = __builtin_bit_cast(uint32_t, __builtin_bit_cast(h16x2, hi) + k);
    return __builtin_amdgcn_perm(b, a, 0x06040200u);
}

// The uint8 side of a tile's C, for closures that keep uint8 data in the
// caller's uint8 matrix and compute on its 16-bit working copy: with kC8In
// the tile's C is read from p (and widened) instead of the working copy, with
// kC8Out the result is also narrowed into p, and with kNo16 it goes to p only;
// kC8Neg complements the uint8 values both ways (255 - v).  p points at the
// tile's first entry, ld in bytes (rows 16-byte aligned).  mode 0: no uint8
// side.
enum { kC8In = 1, kC8Out = 2, kNo16 = 4, kC8Neg = 8 };
struct C8 {
    uint8_t *p;
    int64_t ld;
    int mode;
    __device__ __forceinline__ C8 at(int64_t row, int64_t col) const {
        return C8{mode ? p + row * ld + col : p, ld, mode};
    }
};

// The A-side operand of a packed pair: S - a (u16) or a - 255 (S8, binary16).
template <bool S8>
__device__ __forceinline__ uint32_t neg_pair(uint32_t a) {
    if (S8) return as_word(as_u(as_h(as_pair(a)) - h16x2{(_Float16)255.0f, (_Float16)255.0f}));
    return ~a;
}
template <bool S8>
__device__ __forceinline__ uint16_t neg_one(uint16_t a) {
    if (S8)
        return __builtin_bit_cast(uint16_t,
                                  (_Float16)(__builtin_bit_cast(_Float16, a) - (_Float16)255.0f));
    return (uint16_t)~a;
}

// B rows are read through the constant address space.  The rows of B used by
// a tile are uniform across the wavefront, and this makes the compiler read
// them with scalar loads (SGPR operands) without having to prove that no
// store in the kernel may alias them.  Where a kernel does write rows it also
// reads this way (the panel phase of the closure), reading an entry's old or
// new value gives the same result because the pivot tile is closed.
#define kconst __attribute__((address_space(4)))

// acc (+)= a (x) b for two entries b of B that share one entry a of A, given
// na = neg_pair / neg_one of a in both halves: v_pk_sub_u16 (clamp) then
// v_pk_max_u16; for S8 v_pk_add_f16 then v_pk_maximum_f16.
template <bool S8>
__device__ __forceinline__ u16x2 step(u16x2 acc, u16x2 b, u16x2 na) {
    if (S8) return as_u(__builtin_elementwise_maximum(as_h(acc), as_h(b) + as_h(na)));
    return __builtin_elementwise_max(acc, __builtin_elementwise_sub_sat(b, na));
}

// Two inner steps at once (S8): the two sums enter the accumulator through one
// v_pk_maximum3_f16.
__device__ __forceinline__ u16x2 step2_s8(u16x2 acc, u16x2 b0, u16x2 na0, u16x2 b1, u16x2 na1) {
    return as_u(__builtin_elementwise_maximum(
        __builtin_elementwise_maximum(as_h(acc), as_h(b0) + as_h(na0)), as_h(b1) + as_h(na1)));
}

// ---------------------------------------------------------------------------
// One wavefront computes C (+)= A * B for a tile of up to 64*TM rows (TM rows
// per lane: lane, lane + 64, ...) and up to 2*NW columns (NW packed pairs per
// row), over K inner steps.
//
// The row of B used at inner step k is the same for all 64 lanes, so its
// words are read with scalar loads and enter each packed instruction as the
// SGPR operand; each of those words serves TM packed updates.  Each lane reads
// only its own rows of A (2*KU bytes per row per KU steps) and forms S - a
// with one XOR per two steps.  The inner loop is therefore one v_pk_sub_u16
// and one v_pk_max_u16 per two updates per lane.
//
// B is always read as whole 2*NW-column segments: the caller guarantees they
// lie inside the (padded) rows.  Columns >= ncols of a segment feed only
// accumulators that are not stored.  FULLC: ncols == 2*NW (whole-vector C
// access); otherwise C is read and written entry-exactly.  Rows >= nrows are
// computed on a valid row and not stored.  nrows, ncols >= 1.  A, B and C rows
// are 16-byte aligned (row strides multiples of 8 entries).
// ---------------------------------------------------------------------------
template <int NW, bool FULLC>
__device__ __forceinline__ void row_load(u16x2 (&acc)[NW], const uint16_t *crow, int ncols) {
    if (FULLC) {
#pragma unroll
        for (int q = 0; q < NW / 4; q++) {
            const uint4 v = reinterpret_cast<const uint4 *>(crow)[q];
            acc[4 * q + 0] = as_pair(v.x);
            acc[4 * q + 1] = as_pair(v.y);
            acc[4 * q + 2] = as_pair(v.z);
            acc[4 * q + 3] = as_pair(v.w);
        }
    } else {
#pragma unroll
        for (int w = 0; w < NW; w++) {
            const uint16_t lo = (2 * w < ncols) ? crow[2 * w] : (uint16_t)0;
            const uint16_t hi = (2 * w + 1 < ncols) ? crow[2 * w + 1] : (uint16_t)0;
            acc[w] = u16x2{lo, hi};
        }
    }
}

template <int NW, bool FULLC>
__device__ __forceinline__ void row_store(const u16x2 (&acc)[NW], uint16_t *crow, int ncols) {
    if (FULLC) {
#pragma unroll
        for (int q = 0; q < NW / 4; q++) {
            uint4 v;
            v.x = as_word(acc[4 * q + 0]);
            v.y = as_word(acc[4 * q + 1]);
            v.z = as_word(acc[4 * q + 2]);
            v.w = as_word(acc[4 * q + 3]);
            reinterpret_cast<uint4 *>(crow)[q] = v;
        }
    } else {
#pragma unroll
        for (int w = 0; w < NW; w++) {
            if (2 * w + 1 < ncols) {
                reinterpret_cast<uint32_t *>(crow)[w] = as_word(acc[w]);
            } else if (2 * w < ncols) {
                crow[2 * w] = acc[w].x;
            }
        }
    }
}

// row_load / row_store on the uint8 side of C (2 NW bytes per row; FULLC
// rows are read and written as whole 16-byte or, for NW = 4, 8-byte words).
template <int NW, bool FULLC>
__device__ __forceinline__ void row_load8(u16x2 (&acc)[NW], const uint8_t *crow, int ncols,
                                          bool neg) {
    if (FULLC) {
        uint32_t w[NW / 2];
        if constexpr (NW >= 8) {
#pragma unroll
            for (int q = 0; q < NW / 8; q++) {
                const uint4 v = reinterpret_cast<const uint4 *>(crow)[q];
                w[4 * q + 0] = v.x;
                w[4 * q + 1] = v.y;
                w[4 * q + 2] = v.z;
                w[4 * q + 3] = v.w;
            }
        } else {
            const uint2 v = *reinterpret_cast<const uint2 *>(crow);
            w[0] = v.x;
            w[1] = v.y;
        }
#pragma unroll
        for (int i = 0; i < NW / 2; i++) {
            uint32_t lo, hi;
            widen4(neg ? ~w[i] : w[i], lo, hi);
            acc[2 * i] = as_pair(lo);
            acc[2 * i + 1] = as_pair(hi);
        }
    } else {
        const uint8_t m = neg ? 0xFF : 0;
#pragma unroll
        for (int w = 0; w < NW; w++) {
            const uint16_t lo = (2 * w < ncols) ? u8_to_work((uint8_t)(crow[2 * w] ^ m)) : (uint16_t)0;
            const uint16_t hi =
                (2 * w + 1 < ncols) ? u8_to_work((uint8_t)(crow[2 * w + 1] ^ m)) : (uint16_t)0;
            acc[w] = u16x2{lo, hi};
        }
    }
}

template <int NW, bool FULLC>
__device__ __forceinline__ void row_store8(const u16x2 (&acc)[NW], uint8_t *crow, int ncols,
                                           bool neg) {
    if (FULLC) {
        uint32_t w[NW / 2];
#pragma unroll
        for (int i = 0; i < NW / 2; i++) {
            w[i] = narrow4(as_word(acc[2 * i]), as_word(acc[2 * i + 1]));
            if (neg) w[i] = ~w[i];
        }
        if constexpr (NW >= 8) {
#pragma unroll
            for (int q = 0; q < NW / 8; q++)
                reinterpret_cast<uint4 *>(crow)[q] =
                    uint4{w[4 * q + 0], w[4 * q + 1], w[4 * q + 2], w[4 * q + 3]};
        } else {
            *reinterpret_cast<uint2 *>(crow) = uint2{w[0], w[1]};
        }
    } else {
        const uint8_t m = neg ? 0xFF : 0;
#pragma unroll
        for (int w = 0; w < NW; w++) {
            if (2 * w < ncols) crow[2 * w] = (uint8_t)(work_to_u8(acc[w].x) ^ m);
            if (2 * w + 1 < ncols) crow[2 * w + 1] = (uint8_t)(work_to_u8(acc[w].y) ^ m);
        }
    }
}

// One wavefront widens an nrows x ncols block (nrows <= 64, lane = row) of
// uint8 data at c8 into its working form at C (16-byte aligned rows on both
// sides, the block's first column a multiple of 8).
__device__ __forceinline__ void widen_block_wave(uint16_t *C, int64_t ldc, const C8 &c8, int nrows,
                                                 int ncols) {
    const int lane = threadIdx.x & 63;
    if (lane >= nrows || ncols <= 0) return;
    const uint8_t *src = c8.p + (int64_t)lane * c8.ld;
    uint16_t *dst = C + (int64_t)lane * ldc;
    const bool neg = c8.mode & kC8Neg;
    for (int c = 0; c < ncols; c += 8) {
        if (c + 8 <= ncols) {
            const uint2 v = *reinterpret_cast<const uint2 *>(src + c);
            uint32_t a, b, e, f;
            widen4(neg ? ~v.x : v.x, a, b);
            widen4(neg ? ~v.y : v.y, e, f);
            *reinterpret_cast<uint4 *>(dst + c) = uint4{a, b, e, f};
        } else {
            for (int j = c; j < ncols; j++) dst[j] = u8_to_work((uint8_t)(neg ? ~src[j] : src[j]));
        }
    }
}

template <int TM, int NW, bool S8, bool FULLC, bool GROUPB = !S8>
__device__ __forceinline__ void wave_tile_body(uint16_t *C, int64_t ldc, const uint16_t *A,
                                               int64_t lda, const uint16_t *B, int64_t ldb,
                                               int nrows, int ncols, int K, bool accumulate,
                                               bool sync_before_store, C8 c8 = C8{nullptr, 0, 0}) {
    static_assert(NW % 4 == 0, "NW must be a multiple of 4");
    const int lane = threadIdx.x & 63;
    int64_t r[TM];
    bool live[TM];
#pragma unroll
    for (int t = 0; t < TM; t++) {
        live[t] = lane + 64 * t < nrows;
        r[t] = live[t] ? lane + 64 * t : 0;
    }
    u16x2 acc[TM][NW];
    // the uint8 side: only the mode and each lane's row pointer stay live
    // across the inner loop
    const int m8 = __builtin_amdgcn_readfirstlane(c8.mode);
    uint8_t *row8[TM];
#pragma unroll
    for (int t = 0; t < TM; t++) row8[t] = m8 ? c8.p + r[t] * c8.ld : nullptr;
#pragma unroll
    for (int t = 0; t < TM; t++) {
        if (accumulate) {
            if (m8 & kC8In)
                row_load8<NW, FULLC>(acc[t], row8[t], ncols, m8 & kC8Neg);
            else
                row_load<NW, FULLC>(acc[t], C + r[t] * ldc, ncols);
        } else {
#pragma unroll
            for (int w = 0; w < NW; w++) acc[t][w] = u16x2{0, 0};
        }
    }

    // A is read in groups of AG = 32 entries per row (64 bytes, four 16-byte
    // loads, issued one group ahead): a lane's loads then cover whole halves
    // of 128-byte lines instead of returning to the same line eight times, as
    // 16-byte loads spread over 64 rows would, with the line long evicted.
    // Inside a group, KU inner steps at a time: their KU rows of B occupy
    // KU * NW = 64 SGPRs (at most), which leaves room for addressing without
    // spilling.
    constexpr int KU = NW >= 32 ? 2 : (NW >= 16 ? 4 : 8);
    constexpr int AG = 32;
    const uint16_t *arow[TM];
#pragma unroll
    for (int t = 0; t < TM; t++) arow[t] = A + r[t] * lda;
    int k = 0;
    if (K >= AG) {
        uint4 anext[TM][AG / 8];
#pragma unroll
        for (int t = 0; t < TM; t++)
#pragma unroll
            for (int q = 0; q < AG / 8; q++) anext[t][q] = reinterpret_cast<const uint4 *>(arow[t])[q];
        for (; k + AG <= K; k += AG) {
            uint32_t na[TM][AG / 2];
#pragma unroll
            for (int t = 0; t < TM; t++)
#pragma unroll
                for (int q = 0; q < AG / 8; q++) {
                    na[t][4 * q + 0] = neg_pair<S8>(anext[t][q].x);
                    na[t][4 * q + 1] = neg_pair<S8>(anext[t][q].y);
                    na[t][4 * q + 2] = neg_pair<S8>(anext[t][q].z);
                    na[t][4 * q + 3] = neg_pair<S8>(anext[t][q].w);
                }
            // The prefetch of the next group below is issued only after the
            // negations above have consumed the current group (empty asm
            // statements, which emit nothing: the first pins each S - a value
            // before the second, a memory barrier, orders the loads after
            // them), so the loads reuse its registers instead of copies.
#pragma unroll
            for (int t = 0; t < TM; t++)
#pragma unroll
                for (int i = 0; i < AG / 2; i++) asm volatile("" : "+v"(na[t][i]));
            asm volatile("" ::: "memory");
            if (k + 2 * AG <= K) {
#pragma unroll
                for (int t = 0; t < TM; t++)
#pragma unroll
                    for (int q = 0; q < AG / 8; q++)
                        anext[t][q] = reinterpret_cast<const uint4 *>(arow[t] + k + AG)[q];
            }
#pragma unroll
            for (int kg = 0; kg < AG; kg += KU) {
                const uint16_t *b0 = B + (int64_t)(k + kg) * ldb;
                if (S8) {
                    // steps kk and kk + 1 (an even pair: one word of na); with
                    // GROUPB the group's B rows are loaded first, as below
                    // (faster in the batched update, slower in the
                    // single-matrix closure's, where it is off)
                    uint32_t bg[GROUPB ? KU : 1][NW];
                    if constexpr (GROUPB) {
#pragma unroll
                        for (int kk = 0; kk < KU; kk++) {
                            const kconst uint32_t *bp =
                                (const kconst uint32_t *)(b0 + kk * ldb);
#pragma unroll
                            for (int w = 0; w < NW; w++) bg[kk][w] = bp[w];
                        }
                    }
#pragma unroll
                    for (int kk = 0; kk < KU; kk += 2) {
                        const kconst uint32_t *br0 = (const kconst uint32_t *)(b0 + kk * ldb);
                        const kconst uint32_t *br1 =
                            (const kconst uint32_t *)(b0 + (kk + 1) * ldb);
#pragma unroll
                        for (int t = 0; t < TM; t++) {
                            const uint32_t n2 = na[t][(kg + kk) >> 1];
                            const u16x2 nv0 = u16x2{(uint16_t)n2, (uint16_t)n2};
                            const u16x2 nv1 = u16x2{(uint16_t)(n2 >> 16), (uint16_t)(n2 >> 16)};
#pragma unroll
                            for (int w = 0; w < NW; w++) {
                                const uint32_t x0 = GROUPB ? bg[kk][w] : br0[w];
                                const uint32_t x1 = GROUPB ? bg[kk + 1][w] : br1[w];
                                acc[t][w] =
                                    step2_s8(acc[t][w], as_pair(x0), nv0, as_pair(x1), nv1);
                            }
                        }
                    }
                } else {
                    // the KU rows of B of this group, all loaded before the
                    // first update (one wait per group instead of one per
                    // step: measured +6 % on the closure's update kernel)
                    uint32_t bg[KU][NW];
#pragma unroll
                    for (int kk = 0; kk < KU; kk++) {
                        const kconst uint32_t *bp = (const kconst uint32_t *)(b0 + kk * ldb);
#pragma unroll
                        for (int w = 0; w < NW; w++) bg[kk][w] = bp[w];
                    }
#pragma unroll
                    for (int kk = 0; kk < KU; kk++) {
                        const uint32_t *brow = bg[kk];
#pragma unroll
                        for (int t = 0; t < TM; t++) {
                            const uint32_t n2 = na[t][(kg + kk) >> 1];
                            const uint16_t n =
                                ((kg + kk) & 1) ? (uint16_t)(n2 >> 16) : (uint16_t)n2;
                            const u16x2 nv = u16x2{n, n};
                            // the products of four words first, then their
                            // (+) into the accumulators: no sub -> max pair is
                            // back to back (which costs a wait state), and
                            // only four temporaries are live
#pragma unroll
                            for (int w0 = 0; w0 < NW; w0 += 4) {
                                u16x2 prod[4];
#pragma unroll
                                for (int w = 0; w < 4; w++)
                                    prod[w] = __builtin_elementwise_sub_sat(as_pair(brow[w0 + w]),
                                                                            nv);
#pragma unroll
                                for (int w = 0; w < 4; w++)
                                    acc[t][w0 + w] =
                                        __builtin_elementwise_max(acc[t][w0 + w], prod[w]);
                            }
                        }
                    }
                }
            }
        }
    }
    for (; k < K; k++) {
        const kconst uint32_t *brow = (const kconst uint32_t *)(B + (int64_t)k * ldb);
#pragma unroll
        for (int t = 0; t < TM; t++) {
            const uint16_t n = neg_one<S8>(arow[t][k]);
            const u16x2 nv = u16x2{n, n};
#pragma unroll
            for (int w = 0; w < NW; w++) acc[t][w] = step<S8>(acc[t][w], as_pair(brow[w]), nv);
        }
    }

    if (sync_before_store) __syncthreads();
#pragma unroll
    for (int t = 0; t < TM; t++) {
        if (!live[t]) continue;
        if (!(m8 & kNo16)) row_store<NW, FULLC>(acc[t], C + r[t] * ldc, ncols);
        if (m8 & kC8Out) row_store8<NW, FULLC>(acc[t], row8[t], ncols, m8 & kC8Neg);
    }
}

// The 8-column fallback of wave_tile below.
template <int TM, bool S8>
__device__ __forceinline__ void wave_tile_narrow(uint16_t *C, int64_t ldc, const uint16_t *A,
                                                 int64_t lda, const uint16_t *B, int64_t ldb,
                                                 int nrows, int ncols, int K, bool accumulate,
                                                 C8 c8 = C8{nullptr, 0, 0}) {
    for (int c = 0; c < ncols; c += 8) {
        const int nc = min(8, ncols - c);
        if (nc == 8)
            wave_tile_body<TM, 4, S8, true>(C + c, ldc, A, lda, B + c, ldb, nrows, 8, K,
                                            accumulate, false, c8.at(0, c));
        else
            wave_tile_body<TM, 4, S8, false>(C + c, ldc, A, lda, B + c, ldb, nrows, nc, K,
                                             accumulate, false, c8.at(0, c));
    }
}

// One wavefront, tile of nrows x ncols at C.  bspan: columns of each B row
// readable from the tile origin (row length ld minus the tile's first
// column).  When a whole 2*NW-column segment fits (the usual case) the tile
// runs as one NW-wide tile; otherwise (the last column chunk of a row whose
// length is not a multiple of 2*NW) it runs as 8-column tiles, whose 16-byte
// segments always fit because rows are padded to 16 bytes.
// With sync_before_store the whole workgroup must call this (it executes one
// barrier), including waves with no rows.  In the 8-column fallback the
// sub-tiles store as they finish and the barrier comes last; a row-panel
// update stays exact under that order because the pivot tile is closed (any
// mix of old and new operand entries gives the same result).
template <int TM, int NW, bool S8, bool GROUPB = !S8>
__device__ __forceinline__ void wave_tile(uint16_t *C, int64_t ldc, const uint16_t *A, int64_t lda,
                                          const uint16_t *B, int64_t ldb, int nrows, int ncols,
                                          int64_t bspan, int K, bool accumulate,
                                          bool sync_before_store, C8 c8 = C8{nullptr, 0, 0}) {
    if (nrows <= 0 || ncols <= 0) {
        if (sync_before_store) __syncthreads();
        return;
    }
    if (bspan >= 2 * NW) {
        if (ncols >= 2 * NW)
            wave_tile_body<TM, NW, S8, true, GROUPB>(C, ldc, A, lda, B, ldb, nrows, 2 * NW, K,
                                                     accumulate, sync_before_store, c8);
        else
            wave_tile_body<TM, NW, S8, false, GROUPB>(C, ldc, A, lda, B, ldb, nrows, ncols, K,
                                                      accumulate, sync_before_store, c8);
        return;
    }
    wave_tile_narrow<TM, S8>(C, ldc, A, lda, B, ldb, nrows, ncols, K, accumulate, c8);
    if (sync_before_store) __syncthreads();
}

// ---------------------------------------------------------------------------
// Warshall closure of one bs x bs tile (bs <= 128) by a 256-thread workgroup,
// the tile held in registers.  Thread (ty, tx) = (t / 16, t % 16) owns rows
// 8ty..8ty+7 and columns 8tx..8tx+7 as 8 x 4 packed pairs.
//
// Step k needs row k and column k of the tile; neither changes during step k
// (T_kk (x) x <= x because T_kk <= S, the multiplicative one), so all 64
// updates of a thread are independent.  Two steps k, k+1 share one barrier:
// the owners publish rows k and k+1 and the column pair (T_ik, T_i,k+1) as
// they are before step k, and every thread forms row k+1 and column k+1 as
// step k leaves them itself --
//   T'_k+1,j = T_k+1,j (+) T_k+1,k (x) T_kj,   T'_i,k+1 = T_i,k+1 (+) T_ik (x) T_k,k+1
// -- then applies step k with row k and column k, and step k+1 with the
// primed row and column.  Two LDS buffer sets alternate, so that publishing
// the next pair cannot overwrite what a slower thread still reads.  Entries
// outside bs x bs are held as 0, the additive zero, and stay 0.
// lds_row: 2 x 2 x 64 words, lds_col: 2 x 128 words.  c8: the tile's uint8
// side (read in place of T with kC8In, written with kC8Out).
// ---------------------------------------------------------------------------
template <bool S8>
__device__ __forceinline__ void tile_closure(uint16_t *T, int64_t ld, int bs, uint32_t *lds_row,
                                             uint32_t *lds_col, C8 c8 = C8{nullptr, 0, 0}) {
    const int t = threadIdx.x;
    const int tx = t & 15, ty = t >> 4;
    u16x2 acc[8][4];
    const int c0 = 8 * tx;
    const bool neg8 = c8.mode & kC8Neg;
#pragma unroll
    for (int i = 0; i < 8; i++) {
        const int row = 8 * ty + i;
        if (row < bs && c0 < bs) {
            uint32_t w4[4];
            if (c8.mode & kC8In) {
                // uint8 side: the 8 bytes at once when all lie inside the
                // tile, else entry by entry (the rest read as 0)
                const uint8_t *src = c8.p + (int64_t)row * c8.ld + c0;
                if (c0 + 8 <= bs) {
                    const uint2 v = *reinterpret_cast<const uint2 *>(src);
                    widen4(neg8 ? ~v.x : v.x, w4[0], w4[1]);
                    widen4(neg8 ? ~v.y : v.y, w4[2], w4[3]);
                } else {
#pragma unroll
                    for (int c = 0; c < 4; c++) {
                        const int j = c0 + 2 * c;
                        const uint32_t lo = j < bs ? u8_to_work((uint8_t)(neg8 ? ~src[2 * c] : src[2 * c])) : 0u;
                        const uint32_t hi =
                            j + 1 < bs ? u8_to_work((uint8_t)(neg8 ? ~src[2 * c + 1] : src[2 * c + 1])) : 0u;
                        w4[c] = lo | (hi << 16);
                    }
                }
            } else {
                const uint4 v = *reinterpret_cast<const uint4 *>(T + (int64_t)row * ld + c0);
                w4[0] = v.x;
                w4[1] = v.y;
                w4[2] = v.z;
                w4[3] = v.w;
            }
#pragma unroll
            for (int c = 0; c < 4; c++) {
                u16x2 p = as_pair(w4[c]);
                if (c0 + 2 * c >= bs) p.x = 0;
                if (c0 + 2 * c + 1 >= bs) p.y = 0;
                acc[i][c] = p;
            }
        } else {
#pragma unroll
            for (int c = 0; c < 4; c++) acc[i][c] = u16x2{0, 0};
        }
    }
    __syncthreads();  // the LDS buffers may still be read from a previous use

    const int nq = (bs + 7) >> 3;
    for (int q = 0; q < nq; q++) {
#pragma unroll
        for (int s = 0; s < 8; s += 2) {
            uint32_t *rb = lds_row + ((s >> 1) & 1) * 128;  // row k: rb[0..63], row k+1: rb[64..127]
            uint32_t *cb = lds_col + ((s >> 1) & 1) * 128;  // (T_ik, T_i,k+1) for row i
            if (ty == q) {
                reinterpret_cast<uint4 *>(rb)[tx] = uint4{as_word(acc[s][0]), as_word(acc[s][1]),
                                                          as_word(acc[s][2]), as_word(acc[s][3])};
                reinterpret_cast<uint4 *>(rb + 64)[tx] =
                    uint4{as_word(acc[s + 1][0]), as_word(acc[s + 1][1]), as_word(acc[s + 1][2]),
                          as_word(acc[s + 1][3])};
            }
            if (tx == q) {
                // columns k, k+1 are the two halves of packed pair s / 2
                reinterpret_cast<uint4 *>(cb)[2 * ty] =
                    uint4{as_word(acc[0][s >> 1]), as_word(acc[1][s >> 1]),
                          as_word(acc[2][s >> 1]), as_word(acc[3][s >> 1])};
                reinterpret_cast<uint4 *>(cb)[2 * ty + 1] =
                    uint4{as_word(acc[4][s >> 1]), as_word(acc[5][s >> 1]),
                          as_word(acc[6][s >> 1]), as_word(acc[7][s >> 1])};
            }
            __syncthreads();
            const int k = 8 * q + s;
            const uint4 r0 = reinterpret_cast<const uint4 *>(rb)[tx];
            const uint4 r1 = reinterpret_cast<const uint4 *>(rb + 64)[tx];
            const uint4 n0 = reinterpret_cast<const uint4 *>(cb)[2 * ty];
            const uint4 n1 = reinterpret_cast<const uint4 *>(cb)[2 * ty + 1];
            // T_k,k+1 (entry k+1 of row k) and T_k+1,k (entry k of row k+1)
            const uint16_t a = reinterpret_cast<const uint16_t *>(rb)[k + 1];
            const uint16_t b = reinterpret_cast<const uint16_t *>(rb + 64)[k];
            const u16x2 rk[4] = {as_pair(r0.x), as_pair(r0.y), as_pair(r0.z), as_pair(r0.w)};
            u16x2 rk1[4] = {as_pair(r1.x), as_pair(r1.y), as_pair(r1.z), as_pair(r1.w)};
            const uint16_t nb = neg_one<S8>(b), na = neg_one<S8>(a);
#pragma unroll
            for (int c = 0; c < 4; c++) rk1[c] = step<S8>(rk1[c], rk[c], u16x2{nb, nb});
            const uint32_t cw[8] = {n0.x, n0.y, n0.z, n0.w, n1.x, n1.y, n1.z, n1.w};
#pragma unroll
            for (int i = 0; i < 8; i++) {
                const u16x2 cp = as_pair(cw[i]);  // (T_ik, T_i,k+1)
                // T'_i,k+1 = T_i,k+1 (+) T_ik (x) T_k,k+1, in the high half
                const u16x2 ck = step<S8>(cp, u16x2{cp.x, cp.x}, u16x2{na, na});
                const uint16_t m0 = neg_one<S8>(cp.x), m1 = neg_one<S8>(ck.y);
#pragma unroll
                for (int c = 0; c < 4; c++) {
                    acc[i][c] = step<S8>(acc[i][c], rk[c], u16x2{m0, m0});
                    acc[i][c] = step<S8>(acc[i][c], rk1[c], u16x2{m1, m1});
                }
            }
        }
    }

#pragma unroll
    for (int i = 0; i < 8; i++) {
        const int row = 8 * ty + i;
        if (row >= bs || c0 >= bs) continue;
        if (c8.mode & kC8Out) {
            uint8_t *d8 = c8.p + (int64_t)row * c8.ld + c0;
            if (c0 + 8 <= bs) {
                uint32_t x = narrow4(as_word(acc[i][0]), as_word(acc[i][1]));
                uint32_t y = narrow4(as_word(acc[i][2]), as_word(acc[i][3]));
                *reinterpret_cast<uint2 *>(d8) = uint2{neg8 ? ~x : x, neg8 ? ~y : y};
            } else {
                const uint8_t m = neg8 ? 0xFF : 0;
#pragma unroll
                for (int c = 0; c < 4; c++) {
                    if (c0 + 2 * c < bs) d8[2 * c] = (uint8_t)(work_to_u8(acc[i][c].x) ^ m);
                    if (c0 + 2 * c + 1 < bs) d8[2 * c + 1] = (uint8_t)(work_to_u8(acc[i][c].y) ^ m);
                }
            }
        }
        if (c8.mode & kNo16) continue;
        uint16_t *dst = T + (int64_t)row * ld + c0;
        if (c0 + 8 <= bs) {
            uint4 v;
            v.x = as_word(acc[i][0]);
            v.y = as_word(acc[i][1]);
            v.z = as_word(acc[i][2]);
            v.w = as_word(acc[i][3]);
            *reinterpret_cast<uint4 *>(dst) = v;
        } else {
#pragma unroll
            for (int c = 0; c < 4; c++) {
                if (c0 + 2 * c < bs) dst[2 * c] = acc[i][c].x;
                if (c0 + 2 * c + 1 < bs) dst[2 * c + 1] = acc[i][c].y;
            }
        }
    }
}

// Number of phase-2 workgroups of a round: row panel (two 32-column chunks
// outside the pivot block each) and column panel (one 64-row chunk each).
constexpr int kPanelNW = 16;  // 32 columns per wave in the panel phase
__host__ __device__ inline void panel_wgs(int64_t D, int k0, int bs, int *n_rowwg, int *n_colwg) {
    const int pcw = 2 * kPanelNW;
    const int64_t nchunk_p = (D + pcw - 1) / pcw;
    const int kpc = (k0 + bs + pcw - 1) / pcw - k0 / pcw;
    *n_rowwg = (int)((nchunk_p - kpc + 1) / 2);
    const int64_t nrch = (D + 63) / 64;
    const int kr = (k0 + bs + 63) / 64 - k0 / 64;
    *n_colwg = (int)(nrch - kr);
}

// Phase 2 of a blocked closure round, one workgroup (id bid).  Workgroups
// [0, n_rowwg) take the row panel: two 64-row halves of
// the pivot rows times two 32-column chunks (the chunks outside the pivot
// block, two per workgroup).  The rest take the column panel: one 64-row chunk
// outside the pivot block times the four 32-column chunks of the pivot block.
// Every panel tile is read and written by one workgroup only, and a barrier
// separates its reads from its writes.
//
// c8 (the whole matrix's uint8 side, at entry (0, 0)): with kC8In each wave
// first widens its own tile from there into T, and a barrier makes the
// workgroup's tiles (which are also its operands: the row panel is its own B,
// the column panel its own A) visible before any is read; kC8Out / kNo16
// apply to the stores.
template <bool S8>
__device__ __forceinline__ void fw_panels_wg(uint16_t *T, int64_t ld, int D, int k0, int bs,
                                             int n_rowwg, int bid, C8 c8 = C8{nullptr, 0, 0}) {
    constexpr int NW = kPanelNW, CW = 2 * NW;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform per wave
    const C8 tio{c8.p, c8.ld, c8.mode & ~kC8In};
    if (bid < n_rowwg) {
        const int kc0 = k0 / CW, kc1 = (k0 + bs + CW - 1) / CW;
        const int cc = 2 * bid + (wave >> 1);
        const int c = cc < kc0 ? cc : cc + (kc1 - kc0);
        const int64_t col0 = (int64_t)c * CW;
        const int rofs = (wave & 1) * 64;
        const int nrows = min(64, bs - rofs);
        const int ncols = (int)min<int64_t>(CW, (int64_t)D - col0);
        const int64_t r0 = (int64_t)k0 + rofs;
        if (c8.mode & kC8In) {
            widen_block_wave(T + r0 * ld + col0, ld, c8.at(r0, col0), nrows, ncols);
            __syncthreads();
        }
        wave_tile<1, NW, S8>(T + r0 * ld + col0, ld, T + r0 * ld + k0, ld,
                             T + (int64_t)k0 * ld + col0, ld, nrows, ncols, ld - col0, bs, true,
                             true, tio.at(r0, col0));
    } else {
        const int kr0 = k0 / 64, kr1 = (k0 + bs + 63) / 64;
        const int rc = bid - n_rowwg;
        const int rchunk = rc < kr0 ? rc : rc + (kr1 - kr0);
        const int64_t row0 = (int64_t)rchunk * 64;
        const int nrows = (int)min<int64_t>(64, (int64_t)D - row0);
        const int cofs = wave * CW;
        const int ncols = min(CW, bs - cofs);
        if (c8.mode & kC8In) {
            widen_block_wave(T + row0 * ld + k0 + cofs, ld, c8.at(row0, k0 + cofs), nrows, ncols);
            __syncthreads();
        }
        wave_tile<1, NW, S8>(T + row0 * ld + k0 + cofs, ld, T + row0 * ld + k0, ld,
                             T + (int64_t)k0 * ld + k0 + cofs, ld, nrows, ncols,
                             ld - k0 - cofs, bs, true, true, tio.at(row0, k0 + cofs));
    }
}

// Phase 3 over a rectangle of tiles: row chunks (64*TM rows) [r_lo, r_hi)
// minus [r_ex0, r_ex1), column chunks (2NW columns) [c_lo, c_hi) minus
// [c_ex0, c_ex1); T_ij (+)= T_iK * T_Kj for pivot block K = [k0, k0 + bs).
// Workgroup (bx, by) of a grid with one column per selected column chunk and
// ceil(rows / 4) rows; the four waves of a workgroup share the column chunk.
struct Rect {
    int r_lo, r_hi, r_ex0, r_ex1, c_lo, c_hi, c_ex0, c_ex1;
};

// FULL: every selected column chunk has all 2NW columns inside D (the
// launcher sends a partial last chunk to a FULL = false launch).
// One wave's tile: selected column chunk csel, selected row chunk rsel
// (wave-uniform).  Out-of-range indices do nothing.
// c8: the whole matrix's uint8 side, at entry (0, 0) (mode 0: none).
template <int TM, int NW, bool S8, bool FULL, bool GROUPB = !S8>
__device__ __forceinline__ void fw_update_wave(uint16_t *T, int64_t ld, int D, int k0, int bs,
                                               const Rect &q, int csel, int rsel,
                                               C8 c8 = C8{nullptr, 0, 0}) {
    constexpr int CW = 2 * NW, RW = 64 * TM;
    int c = q.c_lo + csel;
    if (c >= q.c_ex0) c += q.c_ex1 - q.c_ex0;
    int rc = q.r_lo + rsel;
    if (rc >= q.r_ex0) rc += q.r_ex1 - q.r_ex0;
    if (rc >= q.r_hi || c >= q.c_hi) return;
    const int64_t row0 = (int64_t)rc * RW, col0 = (int64_t)c * CW;
    const int nrows = (int)min<int64_t>(RW, (int64_t)D - row0);
    if (FULL) {
        wave_tile_body<TM, NW, S8, true, GROUPB>(T + row0 * ld + col0, ld, T + row0 * ld + k0,
                                                 ld, T + (int64_t)k0 * ld + col0, ld, nrows, CW,
                                                 bs, true, false, c8.at(row0, col0));
    } else {
        const int ncols = (int)min<int64_t>(CW, (int64_t)D - col0);
        wave_tile<TM, NW, S8, GROUPB>(T + row0 * ld + col0, ld, T + row0 * ld + k0, ld,
                                      T + (int64_t)k0 * ld + col0, ld, nrows, ncols, ld - col0, bs,
                                      true, false, c8.at(row0, col0));
    }
}

template <int TM, int NW, bool S8, bool FULL>
__device__ __forceinline__ void fw_update_wg(uint16_t *T, int64_t ld, int D, int k0, int bs,
                                             const Rect &q, int bx, int by) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform per wave
    fw_update_wave<TM, NW, S8, FULL>(T, ld, D, k0, bs, q, bx, by * 4 + wave);
}

}  // namespace dev
}  // namespace sr
