/*
 * semiring.h -- C ABI of libsemiring, the MI355X (gfx950) implementation of
 * the semiring matrix product and transitive closure of
 *
 *   M. de Bondt, "Fast algorithms for anti-distance matrices as a
 *   generalization of Boolean matrices", arXiv 1705.08743.
 *
 * Three semirings (and the distance dual) are supported, as the paper
 * defines them:
 *
 *   SR_BOOL            Boolean matrices (Sec. II): entries {0, 1},
 *                      a (+) b = max(a, b), a (x) b = min(a, b).
 *   SR_ANTIDIST_U8     anti-distance matrices (Sec. III), integer-scaled as in
 *   SR_ANTIDIST_U16    Sec. IV to {0, 1, ..., S} with S = 2^8 - 1 (uint8),
 *   SR_ANTIDIST_U32    2^16 - 1 (uint16) or 2^32 - 1 (uint32):
 *                      a (+) b = max(a, b) and
 *                      a (x) b = max(a + b - S, 0).  Entry S - w encodes a
 *                      distance w; 0 is "no path" (distance >= S saturates).
 *   SR_DISTANCE_U8     distance matrices, the dual the paper adds beside
 *   SR_DISTANCE_U16    anti-distance matrices (its section on distance
 *   SR_DISTANCE_U32
 *                      matrices): entries 0..S hold a distance, S is "no
 *                      path"; a (+) b = min(a, b) and a (x) b = min(a + b, S)
 *                      ("funny" multiplication; the zero matrix is all S).
 *                      By the De Morgan laws stated there, not(A + B) =
 *                      (not A) (x) (not B) with not a = S - a, so these kinds
 *                      run the anti-distance kernels between two entrywise
 *                      complements.
 *
 * Matrix (+) is entrywise; the product is (A*B)_ij = (+)_k A_ik (x) B_kj
 * (Sec. II), evaluated as a running (+) of column-times-row products; the
 * closure is Warshall's / Floyd's algorithm (Sec. II, Sec. III), i.e. the
 * transitive (not reflexive) closure A (+) A*A (+) A*A*A (+) ...
 * (eq. trcl).  Every result is exact integer arithmetic, unique and
 * independent of launch configuration.
 *
 * Memory layout (all matrices row-major, caller-owned device memory):
 *   anti-distance: element (r, c) at base[r * ld + c], ld in ELEMENTS.
 *   Boolean:       bit-packed 64-bit words; entry (r, c) is bit (c % 64) of
 *                  word base[r * ld + c / 64] (least significant bit first,
 *                  the byte/bit order of the paper's Boolean listing,
 *                  Sec. IV); ld in 64-bit WORDS.  Bits at columns >= the
 *                  matrix width ("padding bits") must be zero on input and
 *                  are left zero on output.
 * Alignment: every base pointer must be 16-byte aligned and every row stride
 * (ld times the element size) a multiple of 16 bytes, else SR_EALIGN.  A
 * buffer must span whole rows: rows * ld elements (words), including the
 * padding of its last row; the kernels read (never write) up to the padded row
 * end.  Row strides that are multiples of 128 bytes take the fastest tiles.
 *
 * Streams and ownership: `stream` is a hipStream_t (NULL = the null stream).
 * Calls are asynchronous and stream-ordered: a zero return means the work was
 * validated and enqueued; device-side faults surface at the caller's next
 * synchronisation.  The library never frees, retains or reallocates caller
 * buffers.  It keeps lazily allocated internal scratch (uint8 working copies,
 * batch descriptors) that sr_shutdown() releases.  The library is not
 * re-entrant for concurrent calls on the SAME stream from several host threads;
 * distinct streams may be driven from distinct threads.
 *
 * Errors: argument errors are detected on the host before anything is
 * enqueued and return a negative SR_E* code; sr_last_error() then returns a
 * thread-local message.  No call aborts the process.
 */
#ifndef SEMIRING_H
#define SEMIRING_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Semiring / storage kind (the `kind` argument of every call). */
typedef enum sr_kind {
    SR_BOOL = 0,          /* Boolean, bit-packed uint64 words */
    SR_ANTIDIST_U8 = 1,   /* anti-distance, uint8 entries, S = 255 */
    SR_ANTIDIST_U16 = 2,  /* anti-distance, uint16 entries, S = 65535 */
    SR_DISTANCE_U8 = 3,   /* distance, uint8 entries, S = 255 = no path */
    SR_DISTANCE_U16 = 4,  /* distance, uint16 entries, S = 65535 = no path */
    SR_ANTIDIST_U32 = 5,  /* anti-distance, uint32 entries, S = 2^32 - 1 */
    SR_DISTANCE_U32 = 6   /* distance, uint32 entries, S = 2^32 - 1 = no path */
} sr_kind;

/* Entrywise operations (the `op` argument of semiring_ewise): the table of
 * entrywise operations in Sec. V, on entry values (any non-Boolean kind) or
 * on bits (SR_BOOL). */
enum {
    SR_EW_AND = 0,  /* min(a, b); Boolean AND */
    SR_EW_OR = 1,   /* max(a, b); Boolean OR */
    SR_EW_XOR = 2,  /* |a - b|; Boolean XOR */
    SR_EW_NOT = 3   /* S - a (B unused); Boolean NOT, padding bits stay zero */
};

/* Return codes. */
enum {
    SR_OK = 0,
    SR_EINVAL = -1,        /* bad kind, negative size, ld < width, NULL with nonzero extent */
    SR_EALIAS = -2,        /* semiring_mul output overlaps an input */
    SR_EALIGN = -3,        /* base or row stride not 16-byte aligned */
    SR_ENOMEM = -4,        /* internal scratch allocation failed */
    SR_EDEVICE = -5,       /* a HIP call or kernel launch failed */
    SR_EUNSUPPORTED = -6   /* flag combination not implemented */
};

/* Flags. */
enum {
    SR_ACCUMULATE = 1u,    /* semiring_mul: C := C (+) A*B instead of C := A*B */
    SR_REFLEXIVE = 2u,     /* closure, closure_batched: return I (+) T (eq. rtc) */
    SR_BOOL_BITWISE = 4u,  /* Boolean: force the word OR-AND kernels */
    SR_BOOL_MFMA = 8u,     /* Boolean semiring_mul, and closure's bulk update: the matrix
                              cores (counts of common bits, thresholded; exact); any other
                              kind: SR_EINVAL */
    SR_SERIAL_PHASES = 16u, /* closure: enqueue every phase on the caller's stream in order, without
                               overlapping the next round's pivot and panels on a second stream */
    SR_BOOL_M4R = 32u,     /* Boolean semiring_mul: the "four Russians" table path */
    SR_CLOSURE_SQUARING = 64u,  /* closure: repeated squaring, A * (I (+) A)^(2^j), 2^j >= D-1 */
    SR_CLOSURE_WARSHALL = 128u, /* closure: the blocked Warshall / Floyd loop */
    SR_CLOSURE_BIG_BLOCKS = 256u /* closure: blocks of 512 pivots closed by squaring (not Boolean) */
};

/*
 * semiring_mul -- C := A * B, or C := C (+) A * B with SR_ACCUMULATE.
 *
 * Defined in Sec. II (product formula and the multiplication algorithm that
 * sums column-times-row products) for Boolean matrices and in Sec. III / IV
 * for anti-distance matrices.  A is R x K (lda), B is K x N (ldb), C is R x N
 * (ldc); ld in elements (anti-distance) or 64-bit words (Boolean).
 * K = 0 gives the zero matrix (or leaves C unchanged with SR_ACCUMULATE).
 * R = 0 or N = 0 is a no-op.  C must not overlap A or B (SR_EALIAS): the
 * product is out of place, and the in-place form with all three operands the
 * same matrix is the closure below.
 * Boolean padding bits of A (columns >= K) and B (columns >= N) must be zero.
 * Boolean without a path flag: the autotuned path for the size class, else
 * SR_BOOL_MFMA when R, K and N are all at least 512, else the word kernels.
 * Boolean with SR_BOOL_MFMA: the same product computed as a product of
 * {0, 1} matrices on the matrix cores -- counts of common set bits, > 0
 * exactly when some A_ik = B_kj = 1 -- with 4-bit float operands (or int8
 * ones when the environment sets SR_MFMA_FORMAT=i8), read straight from the
 * packed bits; it takes stream-ordered working memory for a bit-transposed
 * copy of B, round_up(N, 128) * round_up(K, 256) / 8 bytes, and cannot be
 * combined with SR_BOOL_BITWISE or SR_BOOL_M4R (SR_EINVAL).
 */
int semiring_mul(int kind, void *C, int64_t ldc, const void *A, int64_t lda,
                 const void *B, int64_t ldb, int64_t R, int64_t K, int64_t N,
                 unsigned flags, void *stream);

/*
 * semiring_add -- C := A (+) B entrywise (Sec. II matrix addition; the `|`
 * operator of the entrywise table in Sec. V): max for anti-distance, OR for
 * Boolean words, min for distances.  All three are R x N.  C may be exactly A
 * or B (same base and ld); any other overlap is SR_EALIAS.
 */
int semiring_add(int kind, void *C, int64_t ldc, const void *A, int64_t lda,
                 const void *B, int64_t ldb, int64_t R, int64_t N, void *stream);

/*
 * semiring_ewise -- C := A op B (or op A for SR_EW_NOT) entrywise, op from
 * the table of entrywise operations in Sec. V (SR_EW_*).  Shapes, strides and
 * aliasing as semiring_add (N in bits for SR_BOOL); for SR_EW_NOT, B and ldb
 * are ignored.  An op outside SR_EW_AND..SR_EW_NOT is SR_EINVAL.
 */
int semiring_ewise(int kind, int op, void *C, int64_t ldc, const void *A, int64_t lda,
                   const void *B, int64_t ldb, int64_t R, int64_t N, void *stream);

/*
 * closure -- in place, T := A (+) A*A (+) A*A*A (+) ... for the D x D matrix
 * A held in T (Sec. II eq. trcl; Warshall's algorithm, Sec. II, which for
 * anti-distance matrices is Floyd's, Sec. III): the transitive, non-reflexive
 * closure, so the diagonal holds "i lies on a cycle" (Boolean), S minus the
 * shortest cycle through i, saturated (anti-distance), or that cycle's
 * length, or S (distance: the paper's dransclose).  D = 0 is a no-op.
 * flags: SR_REFLEXIVE (I (+) T, eq. rtc: diagonal 1, S, or 0 for distances --
 * the paper's transclosure / dransclosure); SR_SERIAL_PHASES (every phase in
 * order on `stream`); at most one method -- SR_CLOSURE_WARSHALL (the blocked
 * loop), SR_CLOSURE_SQUARING (A * (I (+) A)^(2^j), 2^j >= D - 1, eq. trcl),
 * SR_CLOSURE_BIG_BLOCKS (the loop over blocks of 512 pivots, each closed by
 * squaring; not Boolean) -- else the autotuned method for D's size class or
 * the built-in size rules; for Boolean matrices at most one of
 * SR_BOOL_BITWISE, SR_BOOL_M4R, SR_BOOL_MFMA (the kernels of the loop's bulk
 * update; by default the matrix cores from 2048 vertices on, the word kernels
 * below).  Every method gives the same matrix.
 * Working memory: the loop on 16-bit, 32-bit and Boolean matrices allocates
 * nothing; uint8 data, squaring, big blocks and SR_BOOL_MFMA take
 * stream-ordered working memory (closure_work_bytes() gives the amount), and
 * on a stream being captured a method chosen by default is one that
 * allocates nothing.  A blocked closure of more than two pivot blocks forks
 * onto a second, library-owned stream of default priority (created by the
 * first such call on `stream`) and joins back before its work completes; the
 * fork and join are events, so the sequence can be captured (call closure()
 * once eagerly on the stream first).
 */
int closure(int kind, void *T, int64_t ldt, int64_t D, unsigned flags, void *stream);

/*
 * closure_work_bytes -- the device working memory, in bytes, that closure()
 * with these arguments would allocate stream-ordered for the duration of the
 * call (0 when the method it takes allocates nothing), by the method it would
 * take now (the autotuning table included; as on a stream that is not being
 * captured).  For footprint accounting by callers that admit work by device
 * memory.  A negative SR_E* code for an invalid kind, size or flags.
 */
int64_t closure_work_bytes(int kind, int64_t D, unsigned flags);

/*
 * closure_noalloc -- closure() without any allocation, for callers that
 * cannot allocate: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, flags, result and errors
 * as closure().  The working memory closure() would allocate (the binary16
 * copy of uint8 data: 2 * D * round_up(D, 64) bytes; the squaring closure's
 * two matrices: 2 * D * round_up(D, 64) * entry bytes + 256, for uint8 data
 * 2-byte entries; a big pivot block's: 2 * 512 * 512 * 2 + 256) comes from a
 * static device array of 32 MiB that each device the library runs on holds
 * until the process ends.  A method chosen by default whose working memory
 * does not fit falls back to the blocked loop; if that still does not fit (a
 * uint8 or uint8-distance matrix above 4096 vertices), or a forced method
 * (SR_CLOSURE_SQUARING, SR_CLOSURE_BIG_BLOCKS) does not, the call returns
 * SR_EINVAL before enqueueing anything.  No stream or event is created either:
 * the second stream of the overlapped schedule is used only if an earlier
 * closure() on the same stream created it, else the phases run in order on
 * `stream`.  Every call on one device shares that device's array (the
 * closure clears what must start at zero): calls whose work overlaps in
 * time on one device race and must be serialized by the caller.
 */
int closure_noalloc(int kind, void *T, int64_t ldt, int64_t D, unsigned flags, void *stream);

/*
 * closure_batched -- `count` independent in-place closures, as closure()
 * applied to each (T[g], ldt[g], D[g]).  The three arrays are HOST arrays of
 * length count; T[g] are device pointers, each obeying the alignment rules
 * above.  Every kind; flags: SR_REFLEXIVE.  The
 * matrices must not overlap each other (SR_EALIAS), D[g] <= 65536; a batch
 * one of whose launches would number more than 2^31 - 4 workgroups (or
 * update waves) is SR_EINVAL, and running out of host memory for its work
 * lists SR_ENOMEM.  The
 * batch runs the blocked Floyd-Warshall of closure() round-synchronously: per
 * round, one pivot, one panels and one update launch cover every graph that
 * still has that round (largest graphs first), so a graph of up to 128
 * vertices is closed by the first pivot launch.  The descriptors and the
 * per-round work lists are built on the host and uploaded stream-ordered
 * (the call returns without waiting); uint8 batches use stream-ordered
 * 16-bit working copies (binary16 values), into which the first round's
 * launches widen the data and from which each graph's last-round launches
 * narrow it back; 32-bit batches run the 32-bit
 * wave tiles of closure() with update tiles of 64 x 32 entries (their only
 * shape).  Boolean graphs of at most 1024 vertices are closed in place on
 * their bit rows (Warshall's loop, one workgroup per graph); larger ones as
 * anti-distance matrices with S = 255 whose entries are 255 for a set bit
 * and 0 otherwise (Sec. III: a set bit stands for distance 0, the entry S,
 * a clear one for distance infinity, the entry 0, and with S = 1 the
 * anti-distance matrices are the Boolean ones; on {0, S} entries max and (x)
 * act as OR and AND), in binary16 working copies, 2 * D[g] *
 * round_up(D[g], 8) bytes per graph; bits past column D[g] - 1 must be zero
 * and stay so.  The rounds are three launches
 * each, which is what synchronizes the whole grid between phases.  The
 * update tiles are 64 x 32 entries unless sr_batch_autotune chose another
 * shape for batches of this class.  For a graph-captured form see the
 * prepared batches below.
 */
int closure_batched(int kind, void *const *T, const int64_t *ldt, const int64_t *D,
                    int64_t count, unsigned flags, void *stream);

/*
 * Prepared batches -- closure_batched split into a one-time preparation and a
 * per-closure launch sequence, for a batch whose matrices are closed again
 * and again (new contents, same matrices and sizes).  The sequence holds
 * kernel launches only, so it can be captured into a HIP graph and the whole
 * batch closed by one graph launch.  The closure computed is closure_batched's.
 *
 * sr_batch_create validates (kind, T, ldt, D, count, flags) as closure_batched
 * does, builds the descriptors and per-round work lists with update tiles of
 * shape `tile` (SR_BATCH_TILE_*; SR_BATCH_TILE_AUTO: the autotuned shape for
 * batches of this class, else 64 x 32; any other value is SR_EINVAL),
 * allocates device memory for them -- and for uint8 batches and Boolean
 * graphs of more than 1024 vertices the 16-bit working copies, 2 * D[g] *
 * round_up(D[g], 8) bytes per graph -- with
 * hipMalloc, uploads
 * them on `stream`, waits for the upload and stores the handle in *out
 * (NULL on error).  The three arrays are copied (the caller may free them);
 * the matrices must stay allocated while the handle is used.  SR_EUNSUPPORTED
 * while `stream` is being captured.
 *
 * sr_batch_run enqueues, on `stream`, the in-place closure of the matrices'
 * current contents: no allocation, copy, memset or host callback.  The
 * current device must be the one the handle was created on (SR_EINVAL).  Runs
 * of one handle must not overlap in time (uint8 and Boolean batches share the
 * working copies).
 *
 * sr_batch_autotune times the batch with each update-tile shape (32-bit
 * batches have one, 64 x 32) on zero
 * matrices of the same sizes (allocated for the purpose; the kernels'
 * runtimes do not depend on the entries), once to warm up and twice more;
 * keeps the fastest in the handle and in the autotuning table under the size
 * classes of the largest D and of count (closure_batched and SR_BATCH_TILE_AUTO
 * then use it), and stores it in *chosen (may be NULL).  It synchronizes
 * `stream` and returns SR_EUNSUPPORTED while that is being captured; the
 * matrices of the batch are not touched.  A new shape's plan is uploaded into
 * a new device allocation: the previous plan's stays allocated, unchanged,
 * until sr_batch_destroy, so a graph captured from an earlier sr_batch_run
 * still replays the closure it captured.
 *
 * sr_batch_tile returns the handle's update-tile shape (SR_BATCH_TILE_*).
 * sr_batch_destroy frees the handle (NULL: no-op); hipFree waits for work in
 * flight, and a graph that captured runs of the handle must not be replayed
 * afterwards.
 */
typedef struct sr_batch sr_batch;
enum {
    SR_BATCH_TILE_AUTO = 0,
    SR_BATCH_TILE_64x16 = 1,
    SR_BATCH_TILE_64x32 = 2,
    SR_BATCH_TILE_64x64 = 3
};
int sr_batch_create(int kind, void *const *T, const int64_t *ldt, const int64_t *D,
                    int64_t count, unsigned flags, int tile, sr_batch **out, void *stream);
int sr_batch_run(sr_batch *batch, void *stream);
int sr_batch_autotune(sr_batch *batch, int *chosen, void *stream);
int sr_batch_tile(const sr_batch *batch);
void sr_batch_destroy(sr_batch *batch);

/*
 * Autotuning (not part of the paper's method: it chooses between exact
 * methods that give identical results).  sr_autotune_closure times each
 * closure method that applies to (kind, D) -- the blocked loop (for Boolean:
 * with the bit-sliced, the four-Russians and the matrix-core update), big
 * pivot blocks of 256, 512, 768 and 1024 vertices, repeated squaring -- on a
 * directed path through all D vertices (the
 * squaring's worst case: it stops early once a squaring changes nothing,
 * while the other methods' runtimes do not depend on the entries; Boolean:
 * a zero matrix), once to warm up and twice more, keeps the
 * fastest for the size class of D (the sizes in (2^(c-1), 2^c]) on the current
 * device, and returns its flags in *chosen (may be NULL).  closure() without a
 * method flag then uses it for every D of that class.  sr_autotune_mul does
 * the same for the Boolean product's paths (SR_BOOL_BITWISE, SR_BOOL_M4R,
 * SR_BOOL_MFMA) per size class of (R, K, N); any other kind returns
 * SR_EUNSUPPORTED.  Both allocate, synchronize `stream` and return
 * SR_EUNSUPPORTED while it is being captured; D in [1, 32768], R, K, N in
 * [1, 65536] (SR_EINVAL otherwise).  sr_autotune_clear forgets every choice.
 * The table is thread-safe and kept per process unless saved (below).
 */
int sr_autotune_closure(int kind, int64_t D, unsigned *chosen, void *stream);
int sr_autotune_mul(int kind, int64_t R, int64_t K, int64_t N, unsigned *chosen, void *stream);
void sr_autotune_clear(void);

/*
 * sr_autotune_save / sr_autotune_load -- the autotuning table as a JSON file
 * (one entry per line; keys: the device architecture name, the operation, the
 * kind and the size classes), so that tuning survives the process: save
 * writes every entry (atomically, through a temporary file), load merges a
 * saved file into the table (entries of other architectures are kept but
 * never match).  SR_EINVAL when the file cannot be written or read.  With the
 * environment variable SR_AUTOTUNE_FILE set, the library loads that file
 * when it first consults the table and rewrites it after every autotuning
 * call.  A tuned big-block closure also keeps its pivot block size (256 to
 * 1024 vertices, measured by sr_autotune_closure) in the table; *chosen
 * carries the method flags only.
 */
int sr_autotune_save(const char *path);
int sr_autotune_load(const char *path);

/*
 * Phase timing (a tracing aid, not part of the paper's method).  While
 * enabled, closure() brackets each launch of its three phases -- the pivot
 * tile, the panels, the update of the remaining tiles -- with a pair of
 * hipEvents recorded on the caller's stream, and notes the launch's
 * algorithmic work in semiring updates (bs^3, 2(D-bs)bs^2 and (D-bs)^2 bs for
 * a pivot block of bs vertices).  sr_profile_read() waits for the recorded
 * events of one (kind, phase), returns the summed elapsed milliseconds, the
 * number of launches and the summed updates, and forgets those records.
 * kind: SR_BOOL or an anti-distance kind (both anti-distance kinds share one
 * record set).  Recording adds a few microseconds per launch.
 */
enum { SR_PHASE_PIVOT = 0, SR_PHASE_PANELS = 1, SR_PHASE_UPDATE = 2 };
int sr_profile_enable(int enable);
int sr_profile_read(int kind, int phase, double *total_ms, int64_t *launches, double *updates);

/* Thread-local message describing the last non-SR_OK return on this thread. */
const char *sr_last_error(void);

/* Library version string. */
const char *sr_version(void);

/* Release internal scratch on every device (call with no work in flight). */
void sr_shutdown(void);

#ifdef __cplusplus
}
#endif

#endif /* SEMIRING_H */
