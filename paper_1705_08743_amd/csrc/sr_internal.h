// Internal interface between the C-ABI front end (sr_api.cpp) and the HIP
// kernel launchers (sr_antidist.hip, sr_antidist32.hip, sr_bool.hip,
// sr_bool_mfma.hip, sr_elementwise.hip, sr_batched.hip), the runtime pieces
// (sr_runtime.cpp) and the autotuning table (sr_tune.cpp).  Every launcher
// enqueues on `stream` and returns the hipError_t of the launch; argument
// validation has already happened.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

namespace sr {

// Anti-distance entries live in 16-bit storage on the device.  `s8` selects
// the saturation distance: false -> S = 65535 (uint16 data), true -> S = 255
// (uint8 data widened into a 16-bit working copy that holds each value as a
// binary16 float; see sr_tiles.h).

// Blocked Floyd-Warshall tile edge for anti-distance closures (elements).
constexpr int kAdBlock = 128;
// Blocked Warshall tile edge for Boolean closures (bits).
constexpr int kBoolBlock = 256;

// C (+)= A * B (accumulate) or C := A * B.  Row strides in elements; every
// row stride is a multiple of 8 elements (16 bytes).  bspan: entries of each
// B row readable from B (default: ldb; smaller when B is a block inside a
// wider matrix whose rows end before B's row stride does).  gate: a device
// int read by every workgroup at its start; 0 there makes the whole launch a
// no-op (nullptr: always run).  prev, flag: when flag is given, every stored
// entry of C is compared with the entry at the same place in prev (same
// layout as C) and *flag is set to 1 if any differs (never cleared).
hipError_t launch_ad_mul(bool s8, uint16_t *C, int64_t ldc, const uint16_t *A, int64_t lda,
                         const uint16_t *B, int64_t ldb, int64_t R, int64_t K, int64_t N,
                         bool accumulate, hipStream_t stream, int64_t bspan = -1,
                         const int *gate = nullptr, const uint16_t *prev = nullptr,
                         int *flag = nullptr);

// Up to four independent 16-bit products C (+)= A * B (no output is another
// product's operand), in one launch where they are small enough to share
// one; bspan as for launch_ad_mul (-1: ldb).
struct MulDesc {
    uint16_t *C;
    const uint16_t *A, *B;
    int64_t ldc, lda, ldb, R, K, N, bspan;
};
hipError_t launch_ad_mul_group(bool s8, const MulDesc *d, int n, bool accumulate,
                               hipStream_t stream);

// In-place closure of the D x D matrix T (16-bit storage).  serial: no
// second stream (every phase in order on `stream`).  aux_create: false to
// use the second stream only if it exists already (no stream or event is
// created; this holds for the other closure launchers too).
hipError_t launch_ad_closure(bool s8, uint16_t *T, int64_t ld, int64_t D, bool serial,
                             hipStream_t stream, bool aux_create = true);

// Anti-distance with uint32 entries and S = 2^32 - 1 (sr_antidist32.hip):
// product (strides in elements, multiples of 4) and in-place closure (serial:
// every phase in order on `stream`, without the second stream).
hipError_t launch_ad32_mul(uint32_t *C, int64_t ldc, const uint32_t *A, int64_t lda,
                           const uint32_t *B, int64_t ldb, int64_t R, int64_t K, int64_t N,
                           bool accumulate, hipStream_t stream, int64_t bspan = -1,
                           const int *gate = nullptr, const uint32_t *prev = nullptr,
                           int *flag = nullptr);
// Up to four independent 32-bit products C (+)= A * B (launch_ad_mul_group
// with 32-bit entries).
struct MulDesc32 {
    uint32_t *C;
    const uint32_t *A, *B;
    int64_t ldc, lda, ldb, R, K, N, bspan;
};
hipError_t launch_ad32_mul_group(const MulDesc32 *d, int n, bool accumulate,
                                 hipStream_t stream);
hipError_t launch_ad32_closure(uint32_t *T, int64_t ld, int64_t D, bool serial,
                               hipStream_t stream, bool aux_create = true);

// Individual phases of one blocked Floyd-Warshall round (for tests/timing).
hipError_t launch_ad_fw_pivot(bool s8, uint16_t *T, int64_t ld, int64_t D, int64_t kb,
                              hipStream_t stream);
hipError_t launch_ad_fw_panels(bool s8, uint16_t *T, int64_t ld, int64_t D, int64_t kb,
                               hipStream_t stream);
hipError_t launch_ad_fw_update(bool s8, uint16_t *T, int64_t ld, int64_t D, int64_t kb,
                               hipStream_t stream);

// uint8 <-> 16-bit working copies (binary16 values) of an R x C block
// (strides in elements).
hipError_t launch_widen_u8(uint16_t *dst, int64_t ldd, const uint8_t *src, int64_t lds,
                           int64_t R, int64_t C, hipStream_t stream);
hipError_t launch_narrow_u8(uint8_t *dst, int64_t ldd, const uint16_t *src, int64_t lds,
                            int64_t R, int64_t C, hipStream_t stream);

// Boolean, bit-packed: strides in 64-bit words (even), widths in bits.
// path: kBoolPathAuto (chosen by size), kBoolPathBitwise (the bit-sliced
// kernels), kBoolPathM4r (the "four Russians" tables) or, for the closure's
// bulk update, kBoolPathMfma (the matrix cores).
enum { kBoolPathAuto = 0, kBoolPathBitwise = 1, kBoolPathM4r = 2, kBoolPathMfma = 3 };

// A rectangle of a Boolean closure's update (phase 3): 64-row chunks
// [r_lo, r_hi) minus [r_ex0, r_ex1), times the 32-bit words [w0a, w0b) and
// [w1a, w1b).
struct BRect {
    int r_lo, r_hi, r_ex0, r_ex1;
    int w0a, w0b, w1a, w1b;
};
hipError_t launch_bool_mul(uint64_t *C, int64_t ldc, const uint64_t *A, int64_t lda,
                           const uint64_t *B, int64_t ldb, int64_t R, int64_t K, int64_t N,
                           bool accumulate, int path, hipStream_t stream);
// path: kBoolPathAuto, or force the bit-sliced (kBoolPathBitwise), the
// four-Russians (kBoolPathM4r) or the matrix-core (kBoolPathMfma) kernels for
// the bulk update; the last needs `work`, bool_mfma_closure_work_bytes(D)
// bytes (256-byte aligned, alive until the work has run).
hipError_t launch_bool_closure(uint64_t *T, int64_t ld, int64_t D, bool serial, int path,
                               hipStream_t stream, bool aux_create = true,
                               void *work = nullptr);
// Boolean product with the "four Russians" tables (sr_bool.hip); `launch_bool_mul`
// chooses between it and the bit-sliced kernel, path forces one.
hipError_t launch_bool_mul_m4r(uint64_t *C, int64_t ldc, const uint64_t *A, int64_t lda,
                               const uint64_t *B, int64_t ldb, int64_t R, int64_t K, int64_t N,
                               bool accumulate, hipStream_t stream);

// Boolean product on the matrix cores (sr_bool_mfma.hip): B bit-transposed
// into `work` (bool_mfma_work_bytes(R, K, N) bytes, 256-byte aligned, alive
// until the work has run), counts of common bits on the matrix cores,
// threshold.
size_t bool_mfma_work_bytes(int64_t R, int64_t K, int64_t N);
hipError_t launch_bool_mul_mfma(uint64_t *C, int64_t ldc, const uint64_t *A, int64_t lda,
                                const uint64_t *B, int64_t ldb, int64_t R, int64_t K, int64_t N,
                                bool accumulate, void *work, hipStream_t stream);
// The closure's bulk update on the matrix cores: PT := the transposed pivot
// rows [k0, k0 + bs) of T (strides in 32-bit words; PT holds half of
// bool_mfma_closure_work_bytes(D) bytes, the closure's working memory being
// two such buffers), then T_ij (|)= T_iK * T_Kj over q.
size_t bool_mfma_closure_work_bytes(int64_t D);
hipError_t launch_bool_pivot_transpose(uint32_t *PT, const uint32_t *T, int64_t ld, int64_t D,
                                       int k0, int bs, hipStream_t stream);
hipError_t launch_bool_fw_update_mfma(uint32_t *T, int64_t ld, int64_t D, int k0,
                                      const BRect &q, const uint32_t *PT, hipStream_t stream);

// Entrywise operations (values of the op argument; the table of Sec. V):
// and = min, or = max, xor = |a - b|, not = S - a; on Boolean words AND, OR,
// XOR, NOT.
enum { EW_AND = 0, EW_OR = 1, EW_XOR = 2, EW_NOT = 3 };
// elem_bytes 1, 2 or 4: entries; 8: Boolean 64-bit words.  Widths N in elements
// (words for Boolean); nbits: bits per Boolean row (Boolean NOT clears the
// bits beyond it).  B is not read for EW_NOT.
hipError_t launch_ewise(int elem_bytes, int op, void *C, int64_t ldc, const void *A, int64_t lda,
                        const void *B, int64_t ldb, int64_t R, int64_t N, int64_t nbits,
                        hipStream_t stream);
// Entrywise (+) (EW_OR).
hipError_t launch_add(int elem_bytes, void *C, int64_t ldc, const void *A, int64_t lda,
                      const void *B, int64_t ldb, int64_t R, int64_t N, hipStream_t stream);
// Diagonal of a D x D matrix: entries := value (elem_bytes 1, 2, 4), or bit i of
// row i set (8).
hipError_t launch_diag(int elem_bytes, void *T, int64_t ld, int64_t D, uint32_t value,
                       hipStream_t stream);
// The two ends of the closure by repeated squaring (entries of es = 2 or 4
// bytes; s8: the binary16 form of uint8 data): P := I (+) T with the change
// flags flags[0 .. nflags) cleared (nflags <= 256); and T := the closure
// from P = (I (+) T)^m, m >= D - 1 (P off the diagonal, the best cycle
// through i on it).  Strides in entries, rows 16-byte aligned.
hipError_t launch_power_prep(int es, void *P, int64_t ldp, const void *T, int64_t ldt, int64_t D,
                             uint32_t one, int *flags, int nflags, hipStream_t st);
hipError_t launch_power_finish(int es, bool s8, void *T, int64_t ldt, const void *P, int64_t ldp,
                               int64_t D, hipStream_t st);
// p[0 .. n) := value (32-bit words): a kernel, not a memset node, so that a
// captured graph replays it faithfully.
hipError_t launch_fill32(uint32_t *p, int64_t n, uint32_t value, hipStream_t stream);

// closure() with its working memory either allocated stream-ordered
// (work == nullptr) or taken from a caller's buffer of work_bytes bytes
// (256-byte aligned), which work() returns once every argument, including the
// size of the working memory, has been checked; then nothing is allocated and
// no stream or event is created.  fn names the entry point in error
// messages.  Returns an SR_* code and sets the thread's error message
// (sr_api.cpp).
// block: the pivot block of the big-block method (0: the tuned or default
// size).
int closure_run(int kind, void *T, int64_t ldt, int64_t D, unsigned flags, void *stream,
                int (*work)(void **), size_t work_bytes, const char *fn, int64_t block = 0);
// Sets the thread's error message (printf format) and returns code.
int report(int code, const char *fmt, ...);

// Batched anti-distance closure.  `host_desc` holds `count` descriptors,
// already ordered largest-first; the launcher uploads them with the plan's
// per-round work lists into `dev_buf` (batch_plan_bytes() bytes, 256-byte
// aligned, owned by the caller and alive until the work has run).
struct BatchDesc {
    uint16_t *T;    // matrix in 16-bit storage (the caller's, or a working copy)
    int64_t ld;     // row stride of T, elements (multiple of 8)
    uint8_t *T8;    // uint8 data: the caller's matrix (widened into T, narrowed
                    // back); Boolean data: the caller's bit rows
    int64_t ld8;    // row stride of T8, bytes (a multiple of 16)
    int32_t D;      // vertices
    int32_t flags;  // kDescBits: a Boolean graph closed on its bit rows (T unused)
    uint32_t *T32;  // 32-bit kinds: the caller's matrix (ld in 32-bit elements)
};
// Boolean batches: graphs of at most kBoolBatchSmall vertices are closed on
// their bit rows, one workgroup per graph, with no working copy (flag
// kDescBits); larger ones in the {0, 255} binary16 working copies.
constexpr int kBoolBatchSmall = 1024;
constexpr int32_t kDescBits = 1;
// One entry of a launch's work list: a graph and its first workgroup (or,
// for the update, first wave tile); a sentinel entry holds the launch's total.
struct BatchItem {
    int32_t graph;
    int32_t first;
};
// One launch of a round: its work list (offset into the plan's item array,
// entries without the sentinel), workgroups and, for the update, wave tiles.
struct BatchLaunch {
    int64_t offset;
    int n_items;
    int n_wg;
    int n_units;
};
// Host-side per-round work lists of a batch (they depend on the sizes and the
// update-tile shape only).  tile: 1, 2, 3 = wave tiles of 64 x 16, 64 x 32,
// 64 x 64 entries (anything else: kBatchTileDefault).
constexpr int kBatchTileDefault = 2;
struct BatchPlan;
// nullptr when host memory runs out or a launch of the batch would hold more
// than 2^31 - 4 workgroups (or update waves).
BatchPlan *batch_plan_create(const BatchDesc *host_desc, int64_t count, int tile);
void batch_plan_destroy(BatchPlan *plan);
int batch_plan_tile(const BatchPlan *plan);
// Bytes of the device image: the descriptors (batch_desc_bytes), then the
// work lists.
size_t batch_plan_bytes(const BatchPlan *plan, int64_t count);
size_t batch_desc_bytes(int64_t count);
// Rounds of the plan, the launch of phase 0 (pivot), 1 (panels) or 2
// (update) of round kb, and the largest graph.
int batch_plan_rounds(const BatchPlan *plan);
BatchLaunch batch_plan_phase(const BatchPlan *plan, int phase, int kb);
int batch_plan_max_d(const BatchPlan *plan);
// Writes that image (batch_plan_bytes() bytes) to host memory at dst.
void batch_plan_image(const BatchPlan *plan, const BatchDesc *host_desc, int64_t count, void *dst);
// dual: the batch holds distance matrices (complemented, S - a, before and
// after the anti-distance closure); reflexive: the diagonal is then set to
// the multiplicative identity (S for anti-distance, 0 for distance, a set bit
// for Boolean).  bits (with s8): the batch holds Boolean matrices, closed as
// the {0, 255} anti-distance matrices of their binary16 working copies.
// wide: 32-bit matrices (T32), by launch_ad32_closure_batched_resident.
hipError_t launch_ad_closure_batched(bool s8, const BatchPlan *plan, const BatchDesc *host_desc,
                                     int64_t count, void *dev_buf, bool dual, bool reflexive,
                                     bool bits, bool wide, hipStream_t stream);
// The same closure with the image already in device memory at dev_buf: kernel
// launches only (no copy, allocation or host callback), so it can be captured
// into a graph and replayed.
hipError_t launch_ad_closure_batched_resident(bool s8, const BatchPlan *plan, int64_t count,
                                              const void *dev_buf, bool dual, bool reflexive,
                                              bool bits, bool wide, hipStream_t stream);
// The 32-bit batch (sr_antidist32.hip): the descriptors' T32 matrices, the
// plan built with update tile 2 (64 x 32 entries), image at dev_buf.
hipError_t launch_ad32_closure_batched_resident(const BatchPlan *plan, int64_t count,
                                                const void *dev_buf, bool dual, bool reflexive,
                                                hipStream_t stream);

// Second stream of a closure (sr_runtime.cpp), one per (device, caller
// stream), created on first use at default priority.  aux_acquire() returns it
// locked (the caller enqueues its whole fork/join sequence, then calls
// aux_release) or nullptr when none can be created -- or, with create =
// false, when none exists yet for this (device, caller stream).
struct Aux {
    hipStream_t stream;
    hipEvent_t ev_main;  // recorded on the caller's stream, waited on by `stream`
    hipEvent_t ev_aux[2];  // recorded on `stream`, waited on by the caller's stream
                           // (two, so that one round's can be waited for after
                           // the next round's has been recorded)
    int device;
    int slot;
};
Aux *aux_acquire(hipStream_t caller, bool create = true);
void aux_release(Aux *a);

// Autotuning table (sr_tune.cpp).  op: kTuneClosure (a = D), kTuneMul
// (a, b, c = R, K, N) or kTuneBatch (a = largest D, b = graphs); the stored
// choice is the flag set (SR_CLOSURE_*, SR_BOOL_*) that reproduces the
// measured-fastest method, or for a batch its update-tile code; 0 = not tuned.
enum { kTuneClosure = 1, kTuneMul = 2, kTuneBatch = 3 };
int size_class(int64_t n);
unsigned tuned_get(int op, int kind, int64_t a, int64_t b, int64_t c);
void tuned_set(int op, int kind, int64_t a, int64_t b, int64_t c, unsigned choice);
void tuned_clear();
// The table as JSON text (every device architecture's entries): tuned_save
// returns 0 on success; tuned_load merges a file written by tuned_save and
// returns the number of entries read, or -1 when the file cannot be read.
// With SR_AUTOTUNE_FILE set, the table is loaded from that file on its first
// use and written back after every tuned_set.
int tuned_save(const char *path);
int tuned_load(const char *path);

// Phase timing (sr_runtime.cpp).  kind: 0 Boolean, 1 anti-distance;
// phase: 0 pivot, 1 panels, 2 update.  units: semiring updates of the launch.
bool prof_on();
void prof_begin(hipStream_t st);
void prof_end(hipStream_t st, int kind, int phase, double units);
int prof_enable(int on);
int prof_read(int kind, int phase, double *ms, int64_t *launches, double *units);

}  // namespace sr
