/* Drives every C function of the oracle on small seeded inputs, for a build
 * with AddressSanitizer and UndefinedBehaviorSanitizer.  Each matrix is
 * allocated to end exactly after its last row's last entry (rows - 1 strides
 * plus one row width), so an access past any row that the definitions do not
 * make, or any signed overflow, stops the run.  Besides running clean, a few
 * cross-checks between independent oracle functions must hold: the
 * closure loops against the per-source path searches, the packed Boolean
 * loops against the byte loops.  Exit status 0 on success. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void o_set_threads(int n);
void o_ad_mul(const int32_t *A, int64_t lda, const int32_t *B, int64_t ldb, int32_t *C,
              int64_t ldc, int64_t R, int64_t K, int64_t N, int32_t S, int accumulate);
void o_ad_closure(int32_t *T, int64_t ld, int64_t D, int32_t S);
void o_dist_mul(const int32_t *A, int64_t lda, const int32_t *B, int64_t ldb, int32_t *C,
                int64_t ldc, int64_t R, int64_t K, int64_t N, int32_t S, int accumulate);
void o_dist_closure(int32_t *T, int64_t ld, int64_t D, int32_t S);
void o_ad_closure_rows(const int32_t *A, int64_t ld, int64_t D, int32_t S, const int64_t *rows,
                       int64_t nrows, int32_t *out);
void o_ad_mul64(const int64_t *A, int64_t lda, const int64_t *B, int64_t ldb, int64_t *C,
                int64_t ldc, int64_t R, int64_t K, int64_t N, int64_t S, int accumulate);
void o_ad_closure_steps64(int64_t *T, int64_t ld, int64_t D, int64_t S, int64_t k_begin,
                          int64_t k_end);
void o_dist_mul64(const int64_t *A, int64_t lda, const int64_t *B, int64_t ldb, int64_t *C,
                  int64_t ldc, int64_t R, int64_t K, int64_t N, int64_t S, int accumulate);
void o_dist_closure64(int64_t *T, int64_t ld, int64_t D, int64_t S);
void o_ad_closure_rows64(const int64_t *A, int64_t ld, int64_t D, int64_t S,
                         const int64_t *rows, int64_t nrows, int64_t *out);
void o_bool_mul(const uint8_t *A, int64_t lda, const uint8_t *B, int64_t ldb, uint8_t *C,
                int64_t ldc, int64_t R, int64_t K, int64_t N, int accumulate);
void o_bool_closure(uint8_t *T, int64_t ld, int64_t D);
void o_bool_mul_words(const uint64_t *A, int64_t lda, const uint64_t *B, int64_t ldb,
                      uint64_t *C, int64_t ldc, int64_t R, int64_t K, int64_t N, int accumulate);
void o_bool_closure_words(uint64_t *T, int64_t ld, int64_t D);
void o_bool_closure_rows_words(const uint64_t *A, int64_t ld, int64_t D, const int64_t *rows,
                               int64_t nrows, uint64_t *out, int64_t ld_out);

static uint64_t g_state = 0x1705087430ull;
static uint32_t rnd(void) {
    g_state = g_state * 6364136223846793005ull + 1442695040888963407ull;
    return (uint32_t)(g_state >> 33);
}

/* rows x cols entries of `size` bytes at stride ld, exactly sized */
static void *mat(int64_t rows, int64_t cols, int64_t ld, size_t size) {
    size_t n = rows > 0 ? (size_t)((rows - 1) * ld + cols) : 0;
    void *p = malloc(n * size + 1);
    memset(p, 0, n * size + 1);
    return p;
}

static int failures = 0;
#define CHECK(c, ...)                  \
    do {                               \
        if (!(c)) {                    \
            fprintf(stderr, __VA_ARGS__); \
            fprintf(stderr, "\n");     \
            failures++;                \
        }                              \
    } while (0)

/* anti-distance entries: 0 with probability 1 - p, else S - w, w in [1, wmax] */
static void fill32(int32_t *A, int64_t R, int64_t C, int64_t ld, int32_t S, int pct, int32_t wmax) {
    for (int64_t i = 0; i < R; i++)
        for (int64_t j = 0; j < C; j++)
            A[i * ld + j] = (int)(rnd() % 100) < pct ? S - (int32_t)(1 + rnd() % (uint32_t)wmax) : 0;
}
static void fill64(int64_t *A, int64_t R, int64_t C, int64_t ld, int64_t S, int pct, int64_t wmax) {
    for (int64_t i = 0; i < R; i++)
        for (int64_t j = 0; j < C; j++)
            A[i * ld + j] = (int)(rnd() % 100) < pct ? S - (int64_t)(1 + rnd() % (uint64_t)wmax) : 0;
}

static void products(void) {
    const int64_t shapes[][3] = {{0, 0, 0}, {1, 1, 1}, {3, 0, 5}, {7, 5, 3}, {13, 29, 17}, {33, 64, 65}};
    for (size_t s = 0; s < sizeof shapes / sizeof shapes[0]; s++) {
        const int64_t R = shapes[s][0], K = shapes[s][1], N = shapes[s][2];
        const int64_t lda = K + 3, ldb = N + 1, ldc = N + 2;
        for (int acc = 0; acc < 2; acc++) {
            const int32_t Ss[2] = {255, 65535};
            for (int t = 0; t < 2; t++) {
                int32_t *A = mat(R, K, lda, 4), *B = mat(K, N, ldb, 4), *C = mat(R, N, ldc, 4);
                fill32(A, R, K, lda, Ss[t], 40, Ss[t]);
                fill32(B, K, N, ldb, Ss[t], 40, Ss[t]);
                fill32(C, R, N, ldc, Ss[t], 20, Ss[t]);
                o_ad_mul(A, lda, B, ldb, C, ldc, R, K, N, Ss[t], acc);
                o_dist_mul(A, lda, B, ldb, C, ldc, R, K, N, Ss[t], acc);
                free(A); free(B); free(C);
            }
            const int64_t S64 = 4294967295ll;
            int64_t *A = mat(R, K, lda, 8), *B = mat(K, N, ldb, 8), *C = mat(R, N, ldc, 8);
            fill64(A, R, K, lda, S64, 40, S64);
            fill64(B, K, N, ldb, S64, 40, S64);
            o_ad_mul64(A, lda, B, ldb, C, ldc, R, K, N, S64, acc);
            o_dist_mul64(A, lda, B, ldb, C, ldc, R, K, N, S64, acc);
            free(A); free(B); free(C);
            /* Boolean: bytes against packed words */
            uint8_t *a = mat(R, K, lda, 1), *b = mat(K, N, ldb, 1), *c = mat(R, N, ldc, 1);
            const int64_t kw = (K + 63) / 64 + 1, nw = (N + 63) / 64 + 1;
            uint64_t *aw = mat(R, kw, kw, 8), *bw = mat(K, nw, nw, 8), *cw = mat(R, nw, nw, 8);
            for (int64_t i = 0; i < R; i++)
                for (int64_t k = 0; k < K; k++)
                    if (rnd() % 5 == 0) { a[i * lda + k] = 1; aw[i * kw + k / 64] |= 1ull << (k % 64); }
            for (int64_t k = 0; k < K; k++)
                for (int64_t j = 0; j < N; j++)
                    if (rnd() % 5 == 0) { b[k * ldb + j] = 1; bw[k * nw + j / 64] |= 1ull << (j % 64); }
            o_bool_mul(a, lda, b, ldb, c, ldc, R, K, N, 0);
            o_bool_mul_words(aw, kw, bw, nw, cw, nw, R, K, N, 0);
            for (int64_t i = 0; i < R; i++)
                for (int64_t j = 0; j < N; j++)
                    CHECK(c[i * ldc + j] == ((cw[i * nw + j / 64] >> (j % 64)) & 1),
                          "bool product bytes vs words differ at (%lld, %lld)", (long long)i, (long long)j);
            free(a); free(b); free(c); free(aw); free(bw); free(cw);
        }
    }
}

static void closures(void) {
    const int64_t sizes[] = {0, 1, 2, 5, 31, 64, 70};
    for (size_t s = 0; s < sizeof sizes / sizeof sizes[0]; s++) {
        const int64_t D = sizes[s], ld = D + 5;
        int64_t *rows = malloc(sizeof(int64_t) * (size_t)(D + 1));
        for (int64_t r = 0; r < D; r++) rows[r] = r;
        const int32_t Ss[2] = {255, 65535};
        for (int t = 0; t < 2; t++) {
            int32_t *A = mat(D, D, ld, 4), *T = mat(D, D, ld, 4), *out = mat(D, D, D, 4);
            fill32(A, D, D, ld, Ss[t], 10, Ss[t] / 4);
            if (D) memcpy(T, A, sizeof(int32_t) * (size_t)((D - 1) * ld + D));
            o_ad_closure(T, ld, D, Ss[t]);
            o_ad_closure_rows(A, ld, D, Ss[t], rows, D, out);
            for (int64_t i = 0; i < D; i++)
                for (int64_t j = 0; j < D; j++)
                    CHECK(T[i * ld + j] == out[i * D + j],
                          "closure loop vs path search differ at S=%d (%lld, %lld)", Ss[t],
                          (long long)i, (long long)j);
            if (D) memcpy(T, A, sizeof(int32_t) * (size_t)((D - 1) * ld + D));
            o_dist_closure(T, ld, D, Ss[t]);
            free(A); free(T); free(out);
        }
        const int64_t S64 = 4294967295ll;
        int64_t *A = mat(D, D, ld, 8), *T = mat(D, D, ld, 8), *out = mat(D, D, D, 8);
        fill64(A, D, D, ld, S64, 10, S64 / 4);
        if (D) memcpy(T, A, sizeof(int64_t) * (size_t)((D - 1) * ld + D));
        o_ad_closure_steps64(T, ld, D, S64, 0, D);
        o_ad_closure_rows64(A, ld, D, S64, rows, D, out);
        for (int64_t i = 0; i < D; i++)
            for (int64_t j = 0; j < D; j++)
                CHECK(T[i * ld + j] == out[i * D + j], "64-bit closure loop vs path search differ");
        if (D) memcpy(T, A, sizeof(int64_t) * (size_t)((D - 1) * ld + D));
        o_dist_closure64(T, ld, D, S64);
        free(A); free(T); free(out);
        /* Boolean closures: bytes, packed words, per-source search */
        const int64_t nw = (D + 63) / 64 + 1;
        uint8_t *b = mat(D, D, ld, 1);
        uint64_t *w = mat(D, nw, nw, 8), *w0 = mat(D, nw, nw, 8), *wr = mat(D, nw, nw, 8);
        for (int64_t i = 0; i < D; i++)
            for (int64_t j = 0; j < D; j++)
                if (rnd() % 29 == 0) { b[i * ld + j] = 1; w[i * nw + j / 64] |= 1ull << (j % 64); }
        if (D) memcpy(w0, w, sizeof(uint64_t) * (size_t)((D - 1) * nw + nw));
        o_bool_closure(b, ld, D);
        o_bool_closure_words(w, nw, D);
        o_bool_closure_rows_words(w0, nw, D, rows, D, wr, nw);
        for (int64_t i = 0; i < D; i++)
            for (int64_t j = 0; j < D; j++) {
                const int x = (int)((w[i * nw + j / 64] >> (j % 64)) & 1);
                CHECK(b[i * ld + j] == x && x == (int)((wr[i * nw + j / 64] >> (j % 64)) & 1),
                      "Boolean closures differ at D=%lld (%lld, %lld)", (long long)D, (long long)i,
                      (long long)j);
            }
        free(b); free(w); free(w0); free(wr); free(rows);
    }
}

int main(void) {
    o_set_threads(2);
    products();
    closures();
    if (failures) {
        fprintf(stderr, "%d check(s) failed\n", failures);
        return 1;
    }
    printf("oracle sanitizer run: ok\n");
    return 0;
}
