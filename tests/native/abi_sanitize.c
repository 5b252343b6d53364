/* Drives the host side of libsemiring -- argument validation, method and
 * working-memory planning, the autotuning table's JSON reader and writer,
 * the error strings -- for a build whose host code carries AddressSanitizer
 * and UndefinedBehaviorSanitizer.  Needs no GPU: every compute call here is
 * refused before anything is enqueued (the pointers are never dereferenced).
 * argv[1]: a scratch directory for autotuning files.  Exit status 0 when
 * every expected return code is seen. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "semiring.h"

static int failures = 0;
#define EXPECT(call, want)                                                              \
    do {                                                                                \
        const long long got_ = (long long)(call);                                       \
        if (got_ != (long long)(want)) {                                                \
            fprintf(stderr, "line %d: %s returned %lld, expected %lld (%s)\n", __LINE__, \
                    #call, got_, (long long)(want), sr_last_error());                   \
            failures++;                                                                 \
        }                                                                               \
    } while (0)

static char *const P = (char *)0x100000; /* a 16-byte aligned address, never read */

static void write_file(const char *path, const char *text) {
    FILE *f = fopen(path, "wb");
    if (!f) {
        perror(path);
        exit(2);
    }
    fwrite(text, 1, strlen(text), f);
    fclose(f);
}

static void validation(void) {
    const int U16 = SR_ANTIDIST_U16;
    EXPECT(semiring_mul(7, P, 8, P + 4096, 8, P + 8192, 8, 4, 4, 4, 0, NULL), SR_EINVAL);
    EXPECT(semiring_mul(U16, P, 8, P + 4096, 8, P + 8192, 8, -1, 4, 4, 0, NULL), SR_EINVAL);
    EXPECT(semiring_mul(U16, P, 4, P + 4096, 8, P + 8192, 8, 4, 4, 8, 0, NULL), SR_EINVAL);
    EXPECT(semiring_mul(U16, NULL, 8, P + 4096, 8, P + 8192, 8, 4, 4, 4, 0, NULL), SR_EINVAL);
    EXPECT(semiring_mul(U16, P + 2, 8, P + 4096, 8, P + 8192, 8, 4, 4, 4, 0, NULL), SR_EALIGN);
    EXPECT(semiring_mul(U16, P, 12, P + 4096, 8, P + 8192, 8, 4, 4, 4, 0, NULL), SR_EALIGN);
    EXPECT(semiring_mul(U16, P, 8, P, 8, P + 8192, 8, 4, 4, 4, 0, NULL), SR_EALIAS);
    EXPECT(semiring_mul(U16, P, 8, P + 4096, 8, P + 16, 8, 4, 4, 4, 0, NULL), SR_EALIAS);
    EXPECT(semiring_mul(U16, P, 8, P + 4096, 8, P + 8192, 8, 4, 4, 4, 0x100, NULL), SR_EINVAL);
    EXPECT(semiring_mul(SR_BOOL, P, 1, P + 4096, 2, P + 8192, 2, 4, 4, 4, 0, NULL), SR_EALIGN);
    EXPECT(semiring_mul(SR_BOOL, P, 2, P + 4096, 2, P + 8192, 2, 4, 4, 4,
                        SR_BOOL_MFMA | SR_BOOL_BITWISE, NULL),
           SR_EINVAL);
    EXPECT(semiring_mul(SR_ANTIDIST_U32, P, 6, P + 4096, 4, P + 8192, 4, 4, 4, 4, 0, NULL),
           SR_EALIGN);
    EXPECT(semiring_mul(U16, NULL, 8, NULL, 8, P, 8, 0, 5, 5, 0, NULL), SR_OK);
    /* sizes whose byte spans overflow 64 bits */
    EXPECT(semiring_mul(U16, P, INT64_MAX / 2, P + 4096, 8, P + 8192, 8, INT64_MAX / 4, 4, 4, 0,
                        NULL) < 0, 1);
    EXPECT(semiring_add(U16, P, 8, P + 4096, 8, P + 8192, 4, 4, 8, NULL), SR_EINVAL);
    EXPECT(semiring_add(U16, P + 16, 8, P, 8, P + 8192, 8, 4, 8, NULL), SR_EALIAS);
    EXPECT(semiring_ewise(U16, 7, P, 8, P + 4096, 8, P + 8192, 8, 4, 4, NULL), SR_EINVAL);
    EXPECT(semiring_ewise(U16, SR_EW_NOT, NULL, 8, NULL, 8, NULL, 8, 0, 4, NULL), SR_OK);
    EXPECT(semiring_ewise(SR_BOOL, SR_EW_XOR, P, 2, P + 16, 2, P + 8192, 2, 4, 64, NULL),
           SR_EALIAS);

    EXPECT(closure(U16, P, 8, -1, 0, NULL), SR_EINVAL);
    EXPECT(closure(U16, P, 4, 8, 0, NULL), SR_EINVAL);
    EXPECT(closure(U16, P + 8, 8, 8, 0, NULL), SR_EALIGN);
    EXPECT(closure(U16, P, 8, 8, 0x400, NULL), SR_EINVAL);
    EXPECT(closure(U16, P, 8, 8, SR_CLOSURE_SQUARING | SR_CLOSURE_WARSHALL, NULL), SR_EINVAL);
    EXPECT(closure(SR_BOOL, P, 2, 8, SR_BOOL_MFMA | SR_BOOL_M4R, NULL), SR_EINVAL);
    EXPECT(closure(SR_BOOL, P, 2, 8, SR_CLOSURE_BIG_BLOCKS, NULL), SR_EUNSUPPORTED);
    EXPECT(closure(U16, P, 8, (int64_t)1 << 40, 0, NULL), SR_EINVAL);
    EXPECT(closure(U16, NULL, 8, 0, 0, NULL), SR_OK);
    EXPECT(closure_noalloc(U16, P, 8, -1, 0, NULL), SR_EINVAL);
    EXPECT(closure_noalloc(U16, P, 8, 8, 0x400, NULL), SR_EINVAL);

    {
        void *ptrs[2] = {P, P + 4096}, *over[2] = {P, P + 64};
        int64_t lds[2] = {8, 8}, dims[2] = {8, 8}, dims2[2] = {8, 9}, blds[2] = {1, 1},
                bdims[2] = {65, 65};
        sr_batch *h = NULL;
        EXPECT(closure_batched(9, ptrs, lds, dims, 2, 0, NULL), SR_EINVAL);
        EXPECT(closure_batched(U16, ptrs, lds, dims, -1, 0, NULL), SR_EINVAL);
        EXPECT(closure_batched(U16, NULL, lds, dims, 2, 0, NULL), SR_EINVAL);
        EXPECT(closure_batched(U16, over, lds, dims, 2, 0, NULL), SR_EALIAS);
        EXPECT(closure_batched(U16, ptrs, lds, dims2, 2, 0, NULL), SR_EINVAL);
        EXPECT(closure_batched(SR_BOOL, ptrs, blds, bdims, 2, 0, NULL), SR_EINVAL);
        EXPECT(closure_batched(U16, NULL, NULL, NULL, 0, 0, NULL), SR_OK);
        EXPECT(sr_batch_create(U16, over, lds, dims, 2, 0, 0, &h, NULL), SR_EALIAS);
        EXPECT(sr_batch_create(U16, ptrs, lds, dims, 2, 0, 9, &h, NULL), SR_EINVAL);
        EXPECT(sr_batch_create(U16, ptrs, lds, dims, 2, 0, 0, NULL, NULL), SR_EINVAL);
        EXPECT(sr_batch_run(NULL, NULL), SR_EINVAL);
        EXPECT(sr_batch_tile(NULL), SR_BATCH_TILE_AUTO);
        sr_batch_destroy(NULL);
    }
}

static void planning(void) {
    const int kinds[] = {SR_BOOL, SR_ANTIDIST_U8, SR_ANTIDIST_U16, SR_DISTANCE_U8,
                         SR_DISTANCE_U16, SR_ANTIDIST_U32, SR_DISTANCE_U32};
    const unsigned flags[] = {0, SR_REFLEXIVE, SR_CLOSURE_SQUARING, SR_CLOSURE_WARSHALL,
                              SR_CLOSURE_BIG_BLOCKS, SR_SERIAL_PHASES, SR_BOOL_MFMA, SR_BOOL_M4R,
                              SR_BOOL_BITWISE};
    const int64_t sizes[] = {0, 1, 63, 64, 191, 192, 700, 704, 705, 1024, 1537, 2048, 3073,
                             8192, 16384, 32768, 32769, -5};
    for (size_t a = 0; a < sizeof kinds / sizeof kinds[0]; a++)
        for (size_t b = 0; b < sizeof flags / sizeof flags[0]; b++)
            for (size_t c = 0; c < sizeof sizes / sizeof sizes[0]; c++) {
                const int64_t w = closure_work_bytes(kinds[a], sizes[c], flags[b]);
                if (sizes[c] < 0 && w >= 0) {
                    fprintf(stderr, "closure_work_bytes(%d, %lld, %u) = %lld\n", kinds[a],
                            (long long)sizes[c], flags[b], (long long)w);
                    failures++;
                }
            }
    EXPECT(closure_work_bytes(SR_ANTIDIST_U16, 600, SR_CLOSURE_WARSHALL), 0);
    EXPECT(closure_work_bytes(9, 10, 0), SR_EINVAL);
}

static void autotune_files(const char *dir) {
    char path[4096], out[4096];
    snprintf(path, sizeof path, "%s/tune_in.json", dir);
    snprintf(out, sizeof out, "%s/tune_out.json", dir);
    sr_autotune_clear();
    write_file(path,
               "{\"format\": \"libsemiring-autotune-1\", \"entries\": [\n"
               "{\"arch\": \"\", \"op\": 1, \"kind\": 2, \"class\": [10, 0, 0], \"choice\": 786688},\n"
               "{\"arch\": \"gfx950\", \"op\": 1, \"kind\": 2, \"class\": [9, 0, 0], \"choice\": 128}\n"
               "]}\n");
    EXPECT(sr_autotune_load(path), SR_OK);
    EXPECT(closure_work_bytes(SR_ANTIDIST_U16, 1000, 0), 2 * 768 * 768 * 2 + 256);
    EXPECT(sr_autotune_save(out), SR_OK);
    sr_autotune_clear();
    EXPECT(sr_autotune_load(out), SR_OK);
    EXPECT(closure_work_bytes(SR_ANTIDIST_U16, 1000, 0), 2 * 768 * 768 * 2 + 256);
    sr_autotune_clear();
    /* malformed files are refused whole or read up to the damage, never past
     * the buffers they are parsed into */
    char longarch[3000];
    memset(longarch, 'x', sizeof longarch - 1);
    longarch[sizeof longarch - 1] = 0;
    char big[4000];
    snprintf(big, sizeof big,
             "{\"format\": \"libsemiring-autotune-1\", \"entries\": [\n"
             "{\"arch\": \"%s\", \"op\": 1, \"kind\": 2, \"class\": [10, 0, 0], \"choice\": 128}\n]}\n",
             longarch);
    const char *bad[] = {
        "",
        "{",
        "{\"format\": \"something-else\", \"entries\": []}\n",
        "{\"format\": \"libsemiring-autotune-1\", \"entries\": [\n{\"arch\": \"",
        "{\"format\": \"libsemiring-autotune-1\", \"entries\": [\n{\"arch\": \"\", \"op\": 1\n",
        "{\"format\": \"libsemiring-autotune-1\", \"entries\": [\n"
        "{\"arch\": \"\", \"op\": 99999999999999999999, \"kind\": -7, \"class\": [-1, 1e9, x], "
        "\"choice\": -1}\n]}\n",
        "{\"format\": \"libsemiring-autotune-1\", \"entries\": [\n"
        "{\"arch\": \"\\\"\", \"op\": 1, \"kind\": 2, \"class\": [10, 0, 0], \"choice\": 64}\n]}\n",
        big,
    };
    for (size_t i = 0; i < sizeof bad / sizeof bad[0]; i++) {
        write_file(path, bad[i]);
        (void)sr_autotune_load(path); /* any return code; no memory error */
        (void)closure_work_bytes(SR_ANTIDIST_U16, 1000, 0);
        sr_autotune_clear();
    }
    snprintf(path, sizeof path, "%s/does_not_exist/tune.json", dir);
    EXPECT(sr_autotune_load(path) != SR_OK, 1);
    EXPECT(sr_autotune_save(path) != SR_OK, 1);
    EXPECT(sr_autotune_load(NULL) != SR_OK, 1);
}

int main(int argc, char **argv) {
    if (argc < 2) {
        fprintf(stderr, "usage: %s scratch-dir\n", argv[0]);
        return 2;
    }
    if (!sr_version() || !sr_last_error()) return 1;
    validation();
    planning();
    autotune_files(argv[1]);
    {
        double ms = 0, upd = 0;
        int64_t n = 0;
        (void)sr_profile_read(SR_ANTIDIST_U16, SR_PHASE_UPDATE, &ms, &n, &upd);
        EXPECT(sr_profile_read(SR_ANTIDIST_U16, 7, &ms, &n, &upd), SR_EINVAL);
    }
    sr_shutdown();
    if (failures) {
        fprintf(stderr, "%d check(s) failed\n", failures);
        return 1;
    }
    printf("host sanitizer run: ok\n");
    return 0;
}
