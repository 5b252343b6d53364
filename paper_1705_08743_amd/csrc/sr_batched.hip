// Batched anti-distance closure: many independent graphs of uneven size,
// closed together by the blocked Floyd-Warshall of sr_antidist.hip run
// round-synchronously across the whole batch.
//
// Round kb is three launches, each covering every graph that still has a
// round kb (a graph of D vertices has ceil(D / kAdBlock) rounds):
//   pivot:  one workgroup per graph closes its pivot tile; for a graph of at
//           most kAdBlock vertices this tile is the whole matrix, so round 0's
//           pivot launch closes all small graphs outright;
//   panels: the phase-2 workgroups of all graphs, back to back;
//   update: the phase-3 workgroups of all graphs, back to back.
// A workgroup finds its graph and its workgroup index inside that graph by a
// binary search over per-graph prefix counts built on the host, then runs
// exactly the workgroup body the single-graph kernels run.  Graphs are sorted
// largest first, so in every launch the longest work is dispatched first.
// Every launch has thousands of workgroups (not one per graph), which keeps
// the large graphs from finishing alone on a few compute units; the update
// and panels launches hand their workgroups to the XCDs in chunks (below).
// uint8 batches are closed in 16-bit working copies (binary16 values), into
// which the rounds' own launches widen the data and from which they narrow it
// back (round_c8 below); Boolean graphs of more than kBoolBatchSmall vertices
// are unpacked into such copies before the rounds and packed after them, and
// smaller ones are closed on their bit rows by one workgroup each
// (k_batch_bool_small).  The launch
// sequence holds no allocation, copy or host callback once the plan is in
// device memory, so it can be captured into a graph.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdlib.h>

#include <algorithm>
#include <new>
#include <vector>

#include "sr_batch_dev.h"
#include "sr_internal.h"
#include "sr_tiles.h"

namespace sr {
namespace {

using bdev::cdesc;
using bdev::citems;
using bdev::find_item;
using bdev::Item;
using bdev::kXcdChunk;
using bdev::rounds_of;
using bdev::update_rect;
using bdev::xcd_order;
using dev::fw_panels_wg;
using dev::Rect;
using dev::tile_closure;

// Update-tile shapes of a batch: a wave's tile is 64 rows (one per lane) x
// 2 NW columns (NW packed pairs), NW indexed by the tile code of
// batch_plan_create (1: 64 x 16, 2: 64 x 32, 3: 64 x 64; entry 0 unused).
constexpr int kTileNW[4] = {16, 8, 16, 32};

// uint8 data (io & kIoU8) stays in the caller's uint8 matrix T8 outside the
// rounds: each entry is widened into the working copy T by the one launch of
// round 0 that first reads it (pivot tile, panels or update), and narrowed
// back by the one launch of the graph's last round that last writes it, so
// the rounds need no separate conversion passes over the batch (kIoNeg:
// complemented on the way, 255 - a, for the distance kind).  The three
// launches of a round cover each graph's entries exactly once: the pivot
// tile, the panels (pivot rows and columns outside it) and the rest.
constexpr int kIoU8 = 1, kIoNeg = 2;

// The uint8 side of graph d in round kb (none for S8 = false, where io is
// 0).  The mode is a run-time value, uniform over a wave: the tile code
// branches on it only around its loads and stores, so one copy of the inner
// loop serves every round.  last_no16: the entries this launch writes in the
// graph's last round are read by no later launch (no 16-bit copy needed).
template <bool S8>
__device__ __forceinline__ dev::C8 round_c8(const BatchDesc &d, int kb, int io, bool last_no16) {
    if (!S8 || !(io & kIoU8)) return dev::C8{nullptr, 0, 0};
    int m = (io & kIoNeg) ? dev::kC8Neg : 0;
    if (kb == 0) m |= dev::kC8In;
    if (kb == rounds_of(d.D) - 1) m |= dev::kC8Out | (last_no16 ? dev::kNo16 : 0);
    return dev::C8{d.T8, d.ld8, m};
}

template <bool S8>
__global__ void __launch_bounds__(256)
k_batch_pivot(const BatchDesc *desc, const Item *items, int kb, int io) {
    __shared__ uint32_t lds_row[2 * 128];
    __shared__ uint32_t lds_col[2 * 128];
    const BatchDesc d = cdesc(desc, citems(items)[blockIdx.x].graph);
    const int k0 = kb * kAdBlock, bs = min(kAdBlock, d.D - k0);
    // a graph of one round: its pivot tile is the whole result
    const dev::C8 c8 = round_c8<S8>(d, kb, io, rounds_of(d.D) == 1);
    tile_closure<S8>(d.T + (int64_t)k0 * d.ld + k0, d.ld, bs, lds_row, lds_col, c8.at(k0, k0));
}

template <bool S8>
__global__ void __launch_bounds__(256)
k_batch_panels(const BatchDesc *desc, const Item *items, int n_items, int kb, int xmap, int io) {
    const int bid = xmap ? xcd_order((int)blockIdx.x, (int)gridDim.x, xmap) : (int)blockIdx.x;
    const int i = find_item(items, n_items, bid);
    const BatchDesc d = cdesc(desc, citems(items)[i].graph);
    const int k0 = kb * kAdBlock, bs = min(kAdBlock, d.D - k0);
    int n_rowwg = 0, n_colwg = 0;
    dev::panel_wgs(d.D, k0, bs, &n_rowwg, &n_colwg);
    const int wg = bid - citems(items)[i].first;
    // (the panels are the update's operands: their 16-bit copy stays)
    fw_panels_wg<S8>(d.T, d.ld, d.D, k0, bs, n_rowwg, wg, round_c8<S8>(d, kb, io, false));
}

// Phase 3: one 64 x 2 NW tile per wave.  The waves of all graphs are
// numbered back to back (a graph's tiles column-chunk major), so a
// workgroup's four waves may belong to different graphs; no wave of the
// launch idles except in the last workgroup.
template <int NW, bool S8>
__global__ void __launch_bounds__(256)
k_batch_update(const BatchDesc *desc, const Item *items, int n_items, int kb, int n_waves,
               int xmap, int io) {
    constexpr int CW = 2 * NW;
    const int bid = xmap ? xcd_order((int)blockIdx.x, (int)gridDim.x, xmap) : (int)blockIdx.x;
    const int gw = bid * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (gw >= n_waves) return;
    const int i = find_item(items, n_items, gw);
    const BatchDesc d = cdesc(desc, citems(items)[i].graph);
    const int k0 = kb * kAdBlock, bs = min(kAdBlock, d.D - k0);
    int nc = 0, nr = 0;
    const Rect q = update_rect(d.D, kb, 64, CW, &nc, &nr);
    const int local = gw - citems(items)[i].first;
    // column-chunk major: consecutive waves (most often the four waves of a
    // workgroup) share a column chunk, so its pivot-row segment B, read through
    // the scalar cache, is fetched once for all of them
    const int rsel = local % nr, csel = local / nr;
    int c = csel;
    if (c >= q.c_ex0) c += q.c_ex1 - q.c_ex0;
    const dev::C8 c8 = round_c8<S8>(d, kb, io, true);
    if ((c + 1) * CW <= d.D) {
        dev::fw_update_wave<1, NW, S8, true, true>(d.T, d.ld, d.D, k0, bs, q, csel, rsel, c8);
    } else if (NW > 8) {
        // the graph's last column chunk, D - c CW < CW columns: computed in
        // 16-column pieces, so that at most 15 computed columns go unstored
        // instead of up to CW - 1 (over 4096 graphs of 32 to 1024 vertices,
        // log-uniform, 64 x 64 tiles with whole-width edges compute 9.7 % more
        // updates than the useful ones, with 16-column edge pieces 5.4 %)
        int rc = rsel;
        if (rc >= q.r_ex0) rc += q.r_ex1 - q.r_ex0;
        const int64_t row0 = (int64_t)rc * 64, col0 = (int64_t)c * CW;
        const int nrows = (int)min<int64_t>(64, (int64_t)d.D - row0);
        const int ncols = (int)((int64_t)d.D - col0);
        for (int j = 0; j < ncols; j += 16)
            dev::wave_tile<1, 8, S8, true>(d.T + row0 * d.ld + col0 + j, d.ld,
                                           d.T + row0 * d.ld + k0, d.ld,
                                           d.T + (int64_t)k0 * d.ld + col0 + j, d.ld, nrows,
                                           min(16, ncols - j), d.ld - col0 - j, bs, true, false,
                                           c8.at(row0, col0 + j));
    } else {
        dev::fw_update_wave<1, NW, S8, false, true>(d.T, d.ld, d.D, k0, bs, q, csel, rsel, c8);
    }
}

// Workgroup (g, y) of the conversion launches below takes rows [32 y, 32 y +
// 32) of graph g (the grid has ceil(max D / 32) rows of workgroups; those past
// a graph's last row exit at once).
constexpr int kConvRows = 32;

// Boolean data (bit c of a row: bit c % 8 of byte c / 8, i.e. bit c % 64 of
// 64-bit word c / 64 on this little-endian device; T8 = the bit rows, ld8 in
// bytes) <-> the binary16 working copy of the anti-distance matrix with S =
// 255 whose entries are 255 for a set bit and 0 otherwise.  On such matrices
// (+) = max and (x) (a + b - 255, floored at 0) stay in {0, 255} and act as OR
// and AND, so the anti-distance closure of the copy is the Boolean closure
// (Boolean matrices are the anti-distance matrices of S = 1, rescaled).
// One byte of bits (8 columns) per thread and step.
__global__ void __launch_bounds__(256) k_batch_unpack(const BatchDesc *desc) {
    const BatchDesc d = desc[blockIdx.x];
    const int64_t r0 = (int64_t)blockIdx.y * kConvRows;
    if (r0 >= d.D || (d.flags & kDescBits)) return;
    const int64_t nr = min<int64_t>(kConvRows, (int64_t)d.D - r0);
    const int64_t gpr = ((int64_t)d.D + 7) >> 3;
    const uint32_t one = dev::u8_to_work(255);
    for (int64_t g = threadIdx.x; g < nr * gpr; g += 256) {
        const int64_t row = r0 + g / gpr, c0 = (g % gpr) * 8;
        const uint32_t bits = d.T8[row * d.ld8 + (c0 >> 3)];
        uint32_t v[8];
#pragma unroll
        for (int i = 0; i < 8; i++) v[i] = (c0 + i < d.D && ((bits >> i) & 1u)) ? one : 0u;
        uint4 o;
        o.x = v[0] | (v[1] << 16);
        o.y = v[2] | (v[3] << 16);
        o.z = v[4] | (v[5] << 16);
        o.w = v[6] | (v[7] << 16);
        *reinterpret_cast<uint4 *>(d.T + row * d.ld + c0) = o;
    }
}

// The way back: a set bit for every nonzero entry of columns < D, one byte per
// thread and step.  Bytes past column D - 1 are not written (their bits are
// zero by the caller's contract and stay so).
__global__ void __launch_bounds__(256) k_batch_pack(const BatchDesc *desc) {
    const BatchDesc d = desc[blockIdx.x];
    const int64_t r0 = (int64_t)blockIdx.y * kConvRows;
    if (r0 >= d.D || (d.flags & kDescBits)) return;
    const int64_t nr = min<int64_t>(kConvRows, (int64_t)d.D - r0);
    const int64_t gpr = ((int64_t)d.D + 7) >> 3;
    for (int64_t g = threadIdx.x; g < nr * gpr; g += 256) {
        const int64_t row = r0 + g / gpr, c0 = (g % gpr) * 8;
        const uint4 w = *reinterpret_cast<const uint4 *>(d.T + row * d.ld + c0);
        const uint32_t ww[4] = {w.x, w.y, w.z, w.w};
        uint32_t b = 0;
#pragma unroll
        for (int i = 0; i < 8; i++) {
            const uint32_t e = (ww[i >> 1] >> (16 * (i & 1))) & 0x7FFFu;  // (a -0 reads as 0)
            if (c0 + i < d.D && e != 0u) b |= 1u << i;
        }
        d.T8[row * d.ld8 + (c0 >> 3)] = (uint8_t)b;
    }
}

// uint16 entries complemented in place (65535 - a), every graph.
__global__ void __launch_bounds__(256) k_batch_not(const BatchDesc *desc) {
    const BatchDesc d = desc[blockIdx.x];
    const int64_t r0 = (int64_t)blockIdx.y * kConvRows;
    if (r0 >= d.D) return;
    const int64_t nr = min<int64_t>(kConvRows, (int64_t)d.D - r0);
    for (int64_t g = threadIdx.x; g < nr * d.D; g += 256) {
        uint16_t *e = d.T + (r0 + g / d.D) * d.ld + (g % d.D);
        *e = (uint16_t)~*e;
    }
}

// Diagonal of every graph := value, on the uint8 (T8) or uint16 (T) matrices.
__global__ void __launch_bounds__(256) k_batch_diag(const BatchDesc *desc, int u8, uint32_t value) {
    const BatchDesc d = desc[blockIdx.x];
    if (d.flags & kDescBits) return;  // set by the in-place Boolean kernel
    for (int64_t i = threadIdx.x; i < d.D; i += 256) {
        if (u8)
            d.T8[i * d.ld8 + i] = (uint8_t)value;
        else
            d.T[i * d.ld + i] = (uint16_t)value;
    }
}

// Boolean graphs of at most 32 NW vertices, closed on their bit rows (Sec. II,
// Warshall's loop on bit-packed rows): one workgroup of 32 NW threads per
// graph, thread t holding row t in NW registers.  Step k ORs row k into every
// row with bit k set; row k is read from LDS, where its owner publishes it
// right after its own update in step k - 1 (two alternating buffers, one
// barrier per step: a buffer is rewritten only after every thread has passed
// the barrier that ends the step reading it).  Rows past D, and the waves
// that hold only such rows, take no part; bits past column D - 1 are zero on
// input and stay so.  reflexive: the diagonal bits are set afterwards.
template <int NW>
__global__ void __launch_bounds__(32 * NW)
k_batch_bool_small(const BatchDesc *desc, const Item *items, int reflexive) {
    __shared__ uint32_t prow[2][NW];
    const BatchDesc d = cdesc(desc, citems(items)[blockIdx.x].graph);
    const int n = d.D;
    const int t = threadIdx.x;
    const bool live_wave = (t & ~63) < n;  // uniform over the wave
    uint32_t *row = reinterpret_cast<uint32_t *>(d.T8 + (int64_t)min(t, n - 1) * d.ld8);
    const int nw = (n + 31) >> 5;  // words holding columns < n
    uint32_t r[NW];
#pragma unroll
    for (int w = 0; w < NW; w++) r[w] = (t < n && w < nw) ? row[w] : 0u;
    if (t == 0) {
#pragma unroll
        for (int w = 0; w < NW; w++) prow[0][w] = r[w];
    }
    __syncthreads();
#pragma unroll
    for (int kw = 0; kw < NW; kw++) {
        if (32 * kw >= n) break;
        const int kn = min(32, n - 32 * kw);
        for (int b = 0; b < kn; b++) {
            const int k = 32 * kw + b;
            if (live_wave) {
                const uint32_t m = (uint32_t)__builtin_amdgcn_sbfe(r[kw], b, 1);
                const uint32_t *pk = prow[k & 1];
#pragma unroll
                for (int w = 0; w < NW; w++) r[w] = __builtin_amdgcn_bitop3_b32(pk[w], m, r[w], 0xEA);
            }
            if (t == k + 1) {
#pragma unroll
                for (int w = 0; w < NW; w++) prow[(k + 1) & 1][w] = r[w];
            }
            __syncthreads();
        }
    }
    if (t >= n) return;
    if (reflexive) {
#pragma unroll
        for (int w = 0; w < NW; w++)
            if (w == (t >> 5)) r[w] |= 1u << (t & 31);
    }
#pragma unroll
    for (int w = 0; w < NW; w++)
        if (w < nw) row[w] = r[w];
}

// Size classes of the small Boolean graphs: words per row (and 32 x that
// threads per workgroup).
constexpr int kBoolSmallNW[6] = {2, 4, 8, 16, 24, 32};
constexpr int kBoolSmallClasses = 6;

int bool_small_class(int D) {
    int c = 0;
    while (c + 1 < kBoolSmallClasses && 32 * kBoolSmallNW[c] < D) c++;
    return c;
}

// Host plan: per round, the three item lists (offsets into one array).
using Launch = BatchLaunch;

}  // namespace

struct BatchPlan {
    int tile;   // update-tile code (1, 2, 3)
    int max_d;  // largest graph closed in rounds (in working copies or in place)
    std::vector<Item> items;
    std::vector<Launch> pivot, panels, update;  // per round
    Launch small[kBoolSmallClasses];  // Boolean graphs closed on their bits, per class
};

namespace {

// false when a launch would number more workgroups (or update waves) than
// fit the 32-bit work lists.
bool build_plan(BatchPlan &p, const BatchDesc *hd, int64_t count) {
    constexpr int64_t kMaxUnits = INT32_MAX - 3;
    const int cw = 2 * kTileNW[p.tile];
    int max_rounds = 0;
    p.max_d = 0;
    // a graph's rounds: none for the Boolean graphs closed on their bits
    auto rounds = [&](int64_t g) { return (hd[g].flags & kDescBits) ? 0 : rounds_of(hd[g].D); };
    for (int64_t g = 0; g < count; g++) {
        max_rounds = std::max(max_rounds, rounds(g));
        if (!(hd[g].flags & kDescBits)) p.max_d = std::max(p.max_d, hd[g].D);
    }
    for (int c = 0; c < kBoolSmallClasses; c++) {
        Launch ls{(int64_t)p.items.size(), 0, 0, 0};
        for (int64_t g = 0; g < count; g++) {
            if (!(hd[g].flags & kDescBits) || hd[g].D <= 0 || bool_small_class(hd[g].D) != c)
                continue;
            p.items.push_back(Item{(int32_t)g, ls.n_wg++});
        }
        ls.n_items = ls.n_wg;
        p.items.push_back(Item{-1, ls.n_wg});
        p.small[c] = ls;
    }
    for (int kb = 0; kb < max_rounds; kb++) {
        // pivot: every graph with a round kb
        Launch lp{(int64_t)p.items.size(), 0, 0, 0};
        for (int64_t g = 0; g < count; g++) {
            if (hd[g].D <= 0 || rounds(g) <= kb) continue;
            if (lp.n_wg >= kMaxUnits) return false;
            p.items.push_back(Item{(int32_t)g, lp.n_wg++});
        }
        lp.n_items = lp.n_wg;
        p.items.push_back(Item{-1, lp.n_wg});
        p.pivot.push_back(lp);
        // panels and update: graphs with more than one round
        Launch la{(int64_t)p.items.size(), 0, 0, 0};
        for (int64_t g = 0; g < count; g++) {
            const int D = hd[g].D;
            if (rounds(g) <= std::max(kb, 1)) continue;
            const int k0 = kb * kAdBlock, bs = std::min(kAdBlock, D - k0);
            int r = 0, c = 0;
            dev::panel_wgs(D, k0, bs, &r, &c);
            if (r + c <= 0) continue;
            if ((int64_t)la.n_wg + r + c > kMaxUnits) return false;
            p.items.push_back(Item{(int32_t)g, la.n_wg});
            la.n_wg += r + c;
            la.n_items++;
        }
        p.items.push_back(Item{-1, la.n_wg});
        p.panels.push_back(la);
        Launch lu{(int64_t)p.items.size(), 0, 0, 0};
        for (int64_t g = 0; g < count; g++) {
            const int D = hd[g].D;
            if (rounds(g) <= std::max(kb, 1)) continue;
            int nc = 0, nr = 0;
            (void)update_rect(D, kb, 64, cw, &nc, &nr);
            const int64_t waves = (int64_t)nc * nr;
            if (waves <= 0) continue;
            if ((int64_t)lu.n_units + waves > kMaxUnits) return false;
            p.items.push_back(Item{(int32_t)g, lu.n_units});
            lu.n_units += waves;
            lu.n_items++;
        }
        p.items.push_back(Item{-1, lu.n_units});
        lu.n_wg = (lu.n_units + 3) / 4;
        p.update.push_back(lu);
    }
    return true;
}

size_t desc_bytes_of(int64_t count) {
    return ((size_t)count * sizeof(BatchDesc) + 255) / 256 * 256;
}

}  // namespace

BatchPlan *batch_plan_create(const BatchDesc *host_desc, int64_t count, int tile) {
    auto *p = new (std::nothrow) BatchPlan;
    if (!p) return nullptr;
    p->tile = tile >= 1 && tile <= 3 ? tile : kBatchTileDefault;
    bool ok = false;
    try {
        ok = build_plan(*p, host_desc, count);
    } catch (const std::bad_alloc &) {
        ok = false;
    }
    if (!ok) {
        delete p;
        return nullptr;
    }
    return p;
}

void batch_plan_destroy(BatchPlan *plan) { delete plan; }

int batch_plan_tile(const BatchPlan *plan) { return plan->tile; }

size_t batch_desc_bytes(int64_t count) { return desc_bytes_of(count); }

int batch_plan_rounds(const BatchPlan *plan) { return (int)plan->pivot.size(); }

BatchLaunch batch_plan_phase(const BatchPlan *plan, int phase, int kb) {
    return phase == 0 ? plan->pivot[kb] : (phase == 1 ? plan->panels[kb] : plan->update[kb]);
}

int batch_plan_max_d(const BatchPlan *plan) { return plan->max_d; }

size_t batch_plan_bytes(const BatchPlan *plan, int64_t count) {
    return desc_bytes_of(count) + plan->items.size() * sizeof(Item);
}

void batch_plan_image(const BatchPlan *plan, const BatchDesc *host_desc, int64_t count, void *dst) {
    char *out = static_cast<char *>(dst);
    std::fill_n(out, batch_plan_bytes(plan, count), (char)0);
    std::copy_n(reinterpret_cast<const char *>(host_desc), (size_t)count * sizeof(BatchDesc), out);
    std::copy_n(reinterpret_cast<const char *>(plan->items.data()),
                plan->items.size() * sizeof(Item), out + desc_bytes_of(count));
}

hipError_t launch_ad_closure_batched_resident(bool s8, const BatchPlan *plan, int64_t count,
                                              const void *dev_buf, bool dual, bool reflexive,
                                              bool bits, bool wide, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    if (wide) return launch_ad32_closure_batched_resident(plan, count, dev_buf, dual, reflexive, st);
    const BatchPlan &p = *plan;
    const BatchDesc *desc = static_cast<const BatchDesc *>(dev_buf);
    const Item *items = reinterpret_cast<const Item *>(static_cast<const char *>(dev_buf) +
                                                       desc_bytes_of(count));
    const unsigned ng = (unsigned)count;
    const dim3 conv(ng, (unsigned)std::max<int64_t>(1, ((int64_t)p.max_d + kConvRows - 1) / kConvRows));
    if (bits) {
        // graphs of at most kBoolBatchSmall vertices: on their bit rows, one
        // launch per size class
        for (int c = 0; c < kBoolSmallClasses; c++) {
            const Launch &l = p.small[c];
            if (l.n_wg <= 0) continue;
            const Item *it = items + l.offset;
            const int rf = reflexive ? 1 : 0;
            switch (kBoolSmallNW[c]) {
                case 2: hipLaunchKernelGGL(k_batch_bool_small<2>, dim3(l.n_wg), dim3(64), 0, st, desc, it, rf); break;
                case 4: hipLaunchKernelGGL(k_batch_bool_small<4>, dim3(l.n_wg), dim3(128), 0, st, desc, it, rf); break;
                case 8: hipLaunchKernelGGL(k_batch_bool_small<8>, dim3(l.n_wg), dim3(256), 0, st, desc, it, rf); break;
                case 16: hipLaunchKernelGGL(k_batch_bool_small<16>, dim3(l.n_wg), dim3(512), 0, st, desc, it, rf); break;
                case 24: hipLaunchKernelGGL(k_batch_bool_small<24>, dim3(l.n_wg), dim3(768), 0, st, desc, it, rf); break;
                default: hipLaunchKernelGGL(k_batch_bool_small<32>, dim3(l.n_wg), dim3(1024), 0, st, desc, it, rf); break;
            }
        }
        if (p.pivot.empty()) return hipGetLastError();  // no graph above kBoolBatchSmall
        hipLaunchKernelGGL(k_batch_unpack, conv, dim3(256), 0, st, desc);
    } else if (dual && !s8)
        hipLaunchKernelGGL(k_batch_not, conv, dim3(256), 0, st, desc);
    // uint8 data: widened and narrowed by the rounds' own launches
    const int io = (s8 && !bits) ? (kIoU8 | (dual ? kIoNeg : 0)) : 0;
    // the update kernel of the plan's tile shape, for 16-bit (S8 = false) or
    // binary16 (S8 = true) working data
    using UpdateFn = void (*)(const BatchDesc *, const Item *, int, int, int, int, int);
    // XCD chunk of the update and panels launches (xcd_order; 0 = the plain
    // order).  64 workgroups measured best for 4096 graphs of 32 to 1024
    // vertices (uint16 16.6 -> 15.8 ms, uint8 15.9 -> 14.3 ms; 4 / 16 / 256
    // in between); the
    // environment variables SR_BATCH_XCD and SR_BATCH_XCDP override them.
    static const int xmap = [] {
        const char *v = getenv("SR_BATCH_XCD");
        return v ? std::max(0, atoi(v)) : kXcdChunk;
    }();
    static const int xmapp = [] {
        const char *v = getenv("SR_BATCH_XCDP");
        return v ? std::max(0, atoi(v)) : kXcdChunk;
    }();
    UpdateFn upd = nullptr;
    switch (p.tile * 2 + (s8 ? 1 : 0)) {
        case 2: upd = k_batch_update<8, false>; break;
        case 3: upd = k_batch_update<8, true>; break;
        case 6: upd = k_batch_update<32, false>; break;
        case 7: upd = k_batch_update<32, true>; break;
        case 5: upd = k_batch_update<16, true>; break;
        default: upd = k_batch_update<16, false>; break;
    }
    hipError_t e;
    for (size_t kb = 0; kb < p.pivot.size(); kb++) {
        const Launch &a = p.pivot[kb], &b = p.panels[kb], &c = p.update[kb];
        if (a.n_wg > 0) {
            if (s8)
                hipLaunchKernelGGL(k_batch_pivot<true>, dim3(a.n_wg), dim3(256), 0, st, desc,
                                   items + a.offset, (int)kb, io);
            else
                hipLaunchKernelGGL(k_batch_pivot<false>, dim3(a.n_wg), dim3(256), 0, st, desc,
                                   items + a.offset, (int)kb, io);
        }
        if (b.n_wg > 0) {
            if (s8)
                hipLaunchKernelGGL(k_batch_panels<true>, dim3(b.n_wg), dim3(256), 0, st, desc,
                                   items + b.offset, b.n_items + 1, (int)kb, xmapp, io);
            else
                hipLaunchKernelGGL(k_batch_panels<false>, dim3(b.n_wg), dim3(256), 0, st, desc,
                                   items + b.offset, b.n_items + 1, (int)kb, xmapp, io);
        }
        if (c.n_wg > 0)
            hipLaunchKernelGGL(upd, dim3(c.n_wg), dim3(256), 0, st, desc, items + c.offset,
                               c.n_items + 1, (int)kb, c.n_units, xmap, io);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (bits) {
        // reflexive: the diagonal of the working copy := 255 (a set bit), then back to bits
        if (reflexive)
            hipLaunchKernelGGL(k_batch_diag, dim3(ng), dim3(256), 0, st, desc, 0,
                               (uint32_t)0x5BF8u /* 255 in binary16 */);
        hipLaunchKernelGGL(k_batch_pack, conv, dim3(256), 0, st, desc);
        return hipGetLastError();
    }
    if (dual && !s8) hipLaunchKernelGGL(k_batch_not, conv, dim3(256), 0, st, desc);
    if (reflexive) {
        // the multiplicative identity's diagonal: S (anti-distance), 0 (distance)
        const uint32_t one = dual ? 0u : (s8 ? 255u : 65535u);
        hipLaunchKernelGGL(k_batch_diag, dim3(ng), dim3(256), 0, st, desc, s8 ? 1 : 0, one);
    }
    return hipGetLastError();
}

hipError_t launch_ad_closure_batched(bool s8, const BatchPlan *plan, const BatchDesc *host_desc,
                                     int64_t count, void *dev_buf, bool dual, bool reflexive,
                                     bool bits, bool wide, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    // host image of the descriptors and item lists; freed by a stream
    // callback once the upload has executed
    auto *img = new std::vector<char>(batch_plan_bytes(plan, count));
    batch_plan_image(plan, host_desc, count, img->data());
    hipError_t e = hipMemcpyAsync(dev_buf, img->data(), img->size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipLaunchHostFunc(st, [](void *q) { delete static_cast<std::vector<char> *>(q); }, img);
    else
        delete img;
    if (e != hipSuccess) return e;
    return launch_ad_closure_batched_resident(s8, plan, count, dev_buf, dual, reflexive, bits,
                                              wide, st);
}

}  // namespace sr
