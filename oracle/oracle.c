/*
 * Oracle for the semiring product and closure of de Bondt, "Fast algorithms
 * for anti-distance matrices as a generalization of Boolean matrices"
 * (arXiv 1705.08743).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code, header or constant with the HIP
 * library.
 *
 * Everything here is a plain loop nest written from the paper's definitions,
 * in the order the paper states them, with no blocking and no vector code:
 *
 *   Boolean semiring (Sec. II):  a (+) b = max(a, b),  a (x) b = min(a, b).
 *   Anti-distance semiring, integer-scaled (Sec. III and Sec. IV):
 *       entries in {0, 1, ..., S};  a (+) b = max(a, b);
 *       a (x) b = max(a + b - S, 0)   (the scaled form of max(a + b - 1, 0)).
 *   Matrix (+): entrywise (+).  Matrix product: (A*B)_ij = (+)_k A_ik (x) B_kj.
 *   Multiplication algorithm (Sec. II): P := 0; for each k, P := P (+) (column
 *       k of A) * (row k of B).
 *   Warshall / Floyd (Sec. II, Sec. III): T := A; for each k,
 *       T := T (+) (column k of T) * (row k of T), in place.
 *
 *   Distance matrices (the dual the paper adds in its section on distance
 *   matrices): entries in {0, 1, ..., S} with S standing for "no path";
 *       addition is min (the wedge of the entrywise table), multiplication
 *       is saturating +: a (x) b = min(a + b, S) ("funny" multiplication);
 *       the additive zero is the all-S matrix.  Warshall's loop with these
 *       operations gives the distance closure (minimum lengths over paths of
 *       at least one edge; minimum loop lengths on the diagonal).
 *
 * Anti-distance arithmetic is done in int32 in the definition form
 * max(a + b - S, 0), deliberately not in the saturating-subtract form the
 * GPU kernels use.  Matrices are passed as int32 (anti-distance) or as
 * unpacked {0,1} bytes (Boolean); the bit-packed entry points use 64-bit
 * words with entry (r, c) at bit c mod 64 of word c / 64 of row r, the
 * least-significant-bit-first order of the paper's Boolean listing (Sec. IV).
 *
 * Optional OpenMP: only the i-loop inside one k step is split over threads.
 * Within step k of Warshall, row k and column k do not change (T_kk (x) x <= x
 * because T_kk <= S, the multiplicative one), so the rows of one step are
 * independent and the result is the same for any thread count.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static int g_threads = 1;

void o_set_threads(int n) { g_threads = n < 1 ? 1 : n; }

int o_get_max_threads(void) {
#ifdef _OPENMP
    return omp_get_num_procs();
#else
    return 1;
#endif
}

int o_has_openmp(void) {
#ifdef _OPENMP
    return 1;
#else
    return 0;
#endif
}

/* Anti-distance multiplication, scaled definition (Sec. III, Sec. IV). */
static inline int32_t ad_times(int32_t a, int32_t b, int32_t S) {
    int32_t t = a + b - S;
    return t > 0 ? t : 0;
}

static inline int32_t imax(int32_t a, int32_t b) { return a > b ? a : b; }

/* ---------------------------------------------------------------------------
 * Anti-distance product, multiplication algorithm of Sec. II with the
 * anti-distance operations of Sec. III:
 *   P := 0 (or C when accumulating); for k: P := P (+) A_{:,k} * B_{k,:}.
 * A is R x K (row stride lda), B is K x N (ldb), C is R x N (ldc), int32.
 * ------------------------------------------------------------------------- */
void o_ad_mul(const int32_t *A, int64_t lda, const int32_t *B, int64_t ldb,
              int32_t *C, int64_t ldc, int64_t R, int64_t K, int64_t N,
              int32_t S, int accumulate) {
    if (!accumulate)
        for (int64_t i = 0; i < R; i++)
            for (int64_t j = 0; j < N; j++) C[i * ldc + j] = 0;
    for (int64_t k = 0; k < K; k++) {
        int64_t i;
#pragma omp parallel for num_threads(g_threads) schedule(static)
        for (i = 0; i < R; i++) {
            int32_t a = A[i * lda + k];
            for (int64_t j = 0; j < N; j++) {
                int32_t v = ad_times(a, B[k * ldb + j], S);
                C[i * ldc + j] = imax(C[i * ldc + j], v);
            }
        }
    }
}

/* Anti-distance Warshall / Floyd (Sec. II algorithm with the Sec. III
 * operations), steps k in [k_begin, k_end) only; the full closure is
 * k_begin = 0, k_end = D.  In place on T (D x D, row stride ld). */
void o_ad_closure_steps(int32_t *T, int64_t ld, int64_t D, int32_t S,
                        int64_t k_begin, int64_t k_end) {
    for (int64_t k = k_begin; k < k_end; k++) {
        int64_t i;
#pragma omp parallel for num_threads(g_threads) schedule(static)
        for (i = 0; i < D; i++) {
            int32_t tik = T[i * ld + k];
            for (int64_t j = 0; j < D; j++) {
                int32_t v = ad_times(tik, T[k * ld + j], S);
                T[i * ld + j] = imax(T[i * ld + j], v);
            }
        }
    }
}

void o_ad_closure(int32_t *T, int64_t ld, int64_t D, int32_t S) {
    o_ad_closure_steps(T, ld, D, S, 0, D);
}

/* ---------------------------------------------------------------------------
 * Distance-matrix product (the dual with min as addition and saturating + as
 * multiplication): P := all-S (or C when accumulating); for k:
 * P := min(P, min(A_{:,k} + B_{k,:}, S)).  int32, same shapes as o_ad_mul.
 * ------------------------------------------------------------------------- */
static inline int32_t dist_times(int32_t a, int32_t b, int32_t S) {
    int32_t t = a + b;
    return t < S ? t : S;
}

static inline int32_t imin(int32_t a, int32_t b) { return a < b ? a : b; }

void o_dist_mul(const int32_t *A, int64_t lda, const int32_t *B, int64_t ldb,
                int32_t *C, int64_t ldc, int64_t R, int64_t K, int64_t N,
                int32_t S, int accumulate) {
    if (!accumulate)
        for (int64_t i = 0; i < R; i++)
            for (int64_t j = 0; j < N; j++) C[i * ldc + j] = S;
    for (int64_t k = 0; k < K; k++) {
        int64_t i;
#pragma omp parallel for num_threads(g_threads) schedule(static)
        for (i = 0; i < R; i++) {
            int32_t a = A[i * lda + k];
            for (int64_t j = 0; j < N; j++) {
                int32_t v = dist_times(a, B[k * ldb + j], S);
                C[i * ldc + j] = imin(C[i * ldc + j], v);
            }
        }
    }
}

/* Distance closure: Warshall's loop with min and saturating +, in place
 * (the distance counterpart of o_ad_closure). */
void o_dist_closure(int32_t *T, int64_t ld, int64_t D, int32_t S) {
    for (int64_t k = 0; k < D; k++) {
        int64_t i;
#pragma omp parallel for num_threads(g_threads) schedule(static)
        for (i = 0; i < D; i++) {
            int32_t tik = T[i * ld + k];
            for (int64_t j = 0; j < D; j++) {
                int32_t v = dist_times(tik, T[k * ld + j], S);
                T[i * ld + j] = imin(T[i * ld + j], v);
            }
        }
    }
}

/* Rows of the anti-distance closure straight from its definition, the sum
 * A (+) A*A (+) A*A*A (+) ... (Sec. II, eq. trcl, with the Sec. III
 * operations): entry (i, j) is the largest product of the entries along a
 * path of at least one edge from i to j.  With entry = S - distance this is
 * S - min(S, shortest distance over paths of >= 1 edge).  Computed per source
 * with a dense Dijkstra on distances, all in int64 before saturating.
 * A: D x D int32 (ld); rows: the sources; out: nrows x D int32. */
void o_ad_closure_rows(const int32_t *A, int64_t ld, int64_t D, int32_t S,
                       const int64_t *rows, int64_t nrows, int32_t *out) {
    int64_t r;
#pragma omp parallel for num_threads(g_threads) schedule(dynamic)
    for (r = 0; r < nrows; r++) {
        int64_t src = rows[r];
        const int64_t INF = INT64_MAX / 4;
        int64_t *dist = (int64_t *)malloc(sizeof(int64_t) * (size_t)D);
        char *done = (char *)calloc((size_t)D, 1);
        /* paths of >= 1 edge: start from the out-edges of src. */
        for (int64_t j = 0; j < D; j++) {
            int32_t a = A[src * ld + j];
            dist[j] = a > 0 ? (int64_t)(S - a) : INF;
        }
        for (int64_t it = 0; it < D; it++) {
            int64_t u = -1;
            for (int64_t j = 0; j < D; j++)
                if (!done[j] && dist[j] < INF && (u < 0 || dist[j] < dist[u])) u = j;
            if (u < 0) break;
            done[u] = 1;
            for (int64_t j = 0; j < D; j++) {
                int32_t a = A[u * ld + j];
                if (a > 0) {
                    int64_t nd = dist[u] + (int64_t)(S - a);
                    if (nd < dist[j]) dist[j] = nd;
                }
            }
        }
        for (int64_t j = 0; j < D; j++) {
            int64_t d = dist[j];
            out[r * D + j] = d >= S ? 0 : (int32_t)(S - d);
        }
        free(dist);
        free(done);
    }
}

/* ---------------------------------------------------------------------------
 * The same anti-distance and distance loops in int64, for S = 2^32 - 1
 * (uint32 entries, Sec. IV's scaling with 32-bit storage), where a + b does
 * not fit in int32.  Same definitions, same order.
 * ------------------------------------------------------------------------- */
static inline int64_t ad_times64(int64_t a, int64_t b, int64_t S) {
    int64_t t = a + b - S;
    return t > 0 ? t : 0;
}

static inline int64_t dist_times64(int64_t a, int64_t b, int64_t S) {
    int64_t t = a + b;
    return t < S ? t : S;
}

void o_ad_mul64(const int64_t *A, int64_t lda, const int64_t *B, int64_t ldb, int64_t *C,
                int64_t ldc, int64_t R, int64_t K, int64_t N, int64_t S, int accumulate) {
    if (!accumulate)
        for (int64_t i = 0; i < R; i++)
            for (int64_t j = 0; j < N; j++) C[i * ldc + j] = 0;
    for (int64_t k = 0; k < K; k++) {
        int64_t i;
#pragma omp parallel for num_threads(g_threads) schedule(static)
        for (i = 0; i < R; i++) {
            int64_t a = A[i * lda + k];
            for (int64_t j = 0; j < N; j++) {
                int64_t v = ad_times64(a, B[k * ldb + j], S);
                if (v > C[i * ldc + j]) C[i * ldc + j] = v;
            }
        }
    }
}

void o_ad_closure_steps64(int64_t *T, int64_t ld, int64_t D, int64_t S, int64_t k_begin,
                          int64_t k_end) {
    for (int64_t k = k_begin; k < k_end; k++) {
        int64_t i;
#pragma omp parallel for num_threads(g_threads) schedule(static)
        for (i = 0; i < D; i++) {
            int64_t tik = T[i * ld + k];
            for (int64_t j = 0; j < D; j++) {
                int64_t v = ad_times64(tik, T[k * ld + j], S);
                if (v > T[i * ld + j]) T[i * ld + j] = v;
            }
        }
    }
}

void o_dist_mul64(const int64_t *A, int64_t lda, const int64_t *B, int64_t ldb, int64_t *C,
                  int64_t ldc, int64_t R, int64_t K, int64_t N, int64_t S, int accumulate) {
    if (!accumulate)
        for (int64_t i = 0; i < R; i++)
            for (int64_t j = 0; j < N; j++) C[i * ldc + j] = S;
    for (int64_t k = 0; k < K; k++) {
        int64_t i;
#pragma omp parallel for num_threads(g_threads) schedule(static)
        for (i = 0; i < R; i++) {
            int64_t a = A[i * lda + k];
            for (int64_t j = 0; j < N; j++) {
                int64_t v = dist_times64(a, B[k * ldb + j], S);
                if (v < C[i * ldc + j]) C[i * ldc + j] = v;
            }
        }
    }
}

void o_dist_closure64(int64_t *T, int64_t ld, int64_t D, int64_t S) {
    for (int64_t k = 0; k < D; k++) {
        int64_t i;
#pragma omp parallel for num_threads(g_threads) schedule(static)
        for (i = 0; i < D; i++) {
            int64_t tik = T[i * ld + k];
            for (int64_t j = 0; j < D; j++) {
                int64_t v = dist_times64(tik, T[k * ld + j], S);
                if (v < T[i * ld + j]) T[i * ld + j] = v;
            }
        }
    }
}

/* Rows of the anti-distance closure from the path definition, int64 entries
 * (as o_ad_closure_rows). */
void o_ad_closure_rows64(const int64_t *A, int64_t ld, int64_t D, int64_t S,
                         const int64_t *rows, int64_t nrows, int64_t *out) {
    int64_t r;
#pragma omp parallel for num_threads(g_threads) schedule(dynamic)
    for (r = 0; r < nrows; r++) {
        int64_t src = rows[r];
        const int64_t INF = INT64_MAX / 4;
        int64_t *dist = (int64_t *)malloc(sizeof(int64_t) * (size_t)D);
        char *done = (char *)calloc((size_t)D, 1);
        for (int64_t j = 0; j < D; j++) {
            int64_t a = A[src * ld + j];
            dist[j] = a > 0 ? S - a : INF;
        }
        for (int64_t it = 0; it < D; it++) {
            int64_t u = -1;
            for (int64_t j = 0; j < D; j++)
                if (!done[j] && dist[j] < INF && (u < 0 || dist[j] < dist[u])) u = j;
            if (u < 0) break;
            done[u] = 1;
            for (int64_t j = 0; j < D; j++) {
                int64_t a = A[u * ld + j];
                if (a > 0 && dist[u] + (S - a) < dist[j]) dist[j] = dist[u] + (S - a);
            }
        }
        for (int64_t j = 0; j < D; j++) out[r * D + j] = dist[j] >= S ? 0 : S - dist[j];
        free(dist);
        free(done);
    }
}

/* ---------------------------------------------------------------------------
 * Boolean product on unpacked {0,1} bytes, from the definition of Sec. II:
 *   (A*B)_ij = max_k min(A_ik, B_kj).
 * ------------------------------------------------------------------------- */
void o_bool_mul(const uint8_t *A, int64_t lda, const uint8_t *B, int64_t ldb,
                uint8_t *C, int64_t ldc, int64_t R, int64_t K, int64_t N,
                int accumulate) {
    int64_t i;
#pragma omp parallel for num_threads(g_threads) schedule(static)
    for (i = 0; i < R; i++) {
        for (int64_t j = 0; j < N; j++) {
            uint8_t acc = accumulate ? C[i * ldc + j] : 0;
            for (int64_t k = 0; k < K; k++) {
                uint8_t a = A[i * lda + k], b = B[k * ldb + j];
                uint8_t m = a < b ? a : b;
                if (m > acc) acc = m;
            }
            C[i * ldc + j] = acc;
        }
    }
}

/* Boolean Warshall on unpacked bytes (Sec. II algorithm), in place. */
void o_bool_closure(uint8_t *T, int64_t ld, int64_t D) {
    for (int64_t k = 0; k < D; k++) {
        int64_t i;
#pragma omp parallel for num_threads(g_threads) schedule(static)
        for (i = 0; i < D; i++) {
            uint8_t tik = T[i * ld + k];
            for (int64_t j = 0; j < D; j++) {
                uint8_t b = T[k * ld + j];
                uint8_t m = tik < b ? tik : b;
                if (m > T[i * ld + j]) T[i * ld + j] = m;
            }
        }
    }
}

/* ---------------------------------------------------------------------------
 * Bit-packed Boolean operations (64 entries per word), for sizes where one
 * byte per entry is too slow.  Same loops, with the inner j-loop done 64
 * entries at a time: when entry (i, k) is 1, row i of the result takes the OR
 * of row k of B, as in the paper's Boolean listing (Sec. IV).
 * ------------------------------------------------------------------------- */
static inline int bit_at(const uint64_t *row, int64_t c) {
    return (int)((row[c >> 6] >> (c & 63)) & 1u);
}

void o_bool_mul_words(const uint64_t *A, int64_t lda, const uint64_t *B,
                      int64_t ldb, uint64_t *C, int64_t ldc, int64_t R,
                      int64_t K, int64_t N, int accumulate) {
    int64_t nw = (N + 63) / 64;
    int64_t i;
#pragma omp parallel for num_threads(g_threads) schedule(static)
    for (i = 0; i < R; i++) {
        uint64_t *ci = C + i * ldc;
        if (!accumulate)
            for (int64_t w = 0; w < nw; w++) ci[w] = 0;
        for (int64_t k = 0; k < K; k++) {
            if (bit_at(A + i * lda, k)) {
                const uint64_t *bk = B + k * ldb;
                for (int64_t w = 0; w < nw; w++) ci[w] |= bk[w];
            }
        }
    }
}

void o_bool_closure_words(uint64_t *T, int64_t ld, int64_t D) {
    int64_t nw = (D + 63) / 64;
    for (int64_t k = 0; k < D; k++) {
        const uint64_t *tk = T + k * ld;
        int64_t i;
#pragma omp parallel for num_threads(g_threads) schedule(static)
        for (i = 0; i < D; i++) {
            uint64_t *ti = T + i * ld;
            if (bit_at(ti, k))
                for (int64_t w = 0; w < nw; w++) ti[w] |= tk[w];
        }
    }
}

/* Rows of the Boolean closure from its definition (eq. trcl): entry (i, j) is
 * 1 iff j can be reached from i along a path of at least one edge.  Breadth-
 * first search per source on the packed matrix; out: nrows x ld_out words. */
void o_bool_closure_rows_words(const uint64_t *A, int64_t ld, int64_t D,
                               const int64_t *rows, int64_t nrows,
                               uint64_t *out, int64_t ld_out) {
    int64_t r;
#pragma omp parallel for num_threads(g_threads) schedule(dynamic)
    for (r = 0; r < nrows; r++) {
        int64_t src = rows[r];
        int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * (size_t)(D + 1));
        uint64_t *seen = out + r * ld_out;
        for (int64_t w = 0; w < ld_out; w++) seen[w] = 0;
        int64_t head = 0, tail = 0;
        /* seed with the out-neighbours of src; src itself is not marked. */
        for (int64_t j = 0; j < D; j++)
            if (bit_at(A + src * ld, j) && !bit_at(seen, j)) {
                seen[j >> 6] |= (uint64_t)1 << (j & 63);
                queue[tail++] = j;
            }
        while (head < tail) {
            int64_t u = queue[head++];
            const uint64_t *au = A + u * ld;
            for (int64_t w = 0; w < (D + 63) / 64; w++) {
                uint64_t fresh = au[w] & ~seen[w];
                for (int b = 0; b < 64 && fresh; b++) {
                    if ((fresh >> b) & 1u) {
                        int64_t j = w * 64 + b;
                        seen[w] |= (uint64_t)1 << b;
                        queue[tail++] = j;
                    }
                }
            }
        }
        free(queue);
    }
}
