// Device side of the batched closures, shared by the 16-bit
// (sr_batched.hip) and 32-bit (sr_antidist32.hip) batch kernels: the lookup
// of a workgroup's graph in a launch's work list, the XCD-aware workgroup
// order and the update rectangle of a round.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sr_internal.h"
#include "sr_tiles.h"  // kconst, Rect

namespace sr {
namespace bdev {

using dev::Rect;

// One entry per graph taking part in a launch; `first` is the graph's first
// workgroup; a sentinel entry holds the launch's total.
using Item = BatchItem;

// The work lists and descriptors are read-only while a launch runs and every
// lookup is uniform over a wavefront, so they are read through the constant
// address space (scalar loads, scalar cache) rather than with vector loads.
__device__ __forceinline__ const kconst Item *citems(const Item *p) {
    return (const kconst Item *)p;
}
__device__ __forceinline__ BatchDesc cdesc(const BatchDesc *desc, int g) {
    const kconst BatchDesc *p = (const kconst BatchDesc *)desc + g;
    BatchDesc d;
    d.T = p->T;
    d.ld = p->ld;
    d.T8 = p->T8;
    d.ld8 = p->ld8;
    d.D = p->D;
    d.flags = p->flags;
    d.T32 = p->T32;
    return d;
}

__device__ __forceinline__ int find_item(const Item *items, int n, int bid) {
    const kconst Item *it = citems(items);
    int lo = 0, hi = n - 1;  // largest i with it[i].first <= bid
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (it[mid].first <= bid)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

__host__ __device__ inline int rounds_of(int D) { return (D + kAdBlock - 1) / kAdBlock; }

// Workgroup bid of a launch of nwg runs on XCD bid % 8 (workgroups are handed
// to the eight XCDs in turn).  The renumbering gives each XCD chunks of g
// consecutive workgroups of the plan (chunk c to XCD c % 8), so that the
// workgroups of one graph mostly run on one XCD and reuse the graph's pivot
// row and column blocks from its L2 -- in the plain order consecutive
// workgroups, most often of the same graph, land on eight different XCDs and
// each L2 fetches the blocks again -- while every XCD still gets an even mix
// of the batch's large and small graphs.  Workgroups past the last whole
// round of 8 chunks keep their number.
constexpr int kXcdChunk = 64;

__device__ __forceinline__ int xcd_order(int bid, int nwg, int g) {
    constexpr int kXcd = 8;
    const int full = nwg / (kXcd * g) * (kXcd * g);
    if (bid >= full) return bid;
    const int x = bid % kXcd, j = bid / kXcd;
    return ((j / g) * kXcd + x) * g + j % g;
}

// The full update rectangle of round kb for a graph of D vertices, in wave
// tiles of RW rows x CW columns.
__host__ __device__ inline Rect update_rect(int D, int kb, int RW, int CW, int *ncols_sel,
                                            int *nrows_sel) {
    const int k0 = kb * kAdBlock, bs = min(kAdBlock, D - k0);
    Rect q;
    q.r_lo = 0;
    q.r_hi = (D + RW - 1) / RW;
    q.r_ex0 = k0 / RW;
    q.r_ex1 = (k0 + bs + RW - 1) / RW;
    q.c_lo = 0;
    q.c_hi = (D + CW - 1) / CW;
    q.c_ex0 = k0 / CW;
    q.c_ex1 = (k0 + bs + CW - 1) / CW;
    *ncols_sel = (q.c_hi - q.c_lo) - (q.c_ex1 - q.c_ex0);
    *nrows_sel = (q.r_hi - q.r_lo) - (q.r_ex1 - q.r_ex0);
    return q;
}

}  // namespace bdev
}  // namespace sr
