/* Host-only exercise of the C-ABI under AddressSanitizer: argument checks on
 * NULL handles and buffers, the launch-tuning cache reader on well-formed,
 * corrupt, oversized and binary input, and the report's truncation. Makes no
 * device call beyond context creation (which fails cleanly without a GPU).
 * usage: asan_driver <scratch directory>; exit status 0 when every check
 * holds (the sanitizer aborts the run on a memory error). */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "gdr.h"

static int fails = 0;
#define CHECK(cond)                                                      \
    do {                                                                 \
        if (!(cond)) {                                                   \
            fprintf(stderr, "check failed line %d: %s\n", __LINE__, #cond); \
            ++fails;                                                     \
        }                                                                \
    } while (0)

static void write_file(const char* path, const char* data, size_t len) {
    FILE* f = fopen(path, "wb");
    if (!f) { perror(path); exit(2); }
    fwrite(data, 1, len, f);
    fclose(f);
}

int main(int argc, char** argv) {
    if (argc < 2) return 2;
    char path[4096];
    gdr_params p;
    gdr_params_default(&p);
    CHECK(p.m_dr > p.k && p.tol > 0);

    /* NULL handles and outputs */
    CHECK(gdr_ctx_create(0, NULL, NULL) == GDR_ERR_ARG);
    CHECK(gdr_op_size(NULL) == 0);
    CHECK(gdr_defl_k(NULL) == -1);
    CHECK(gdr_op_link_bytes(NULL, 0) == -1);
    gdr_c64 s = {0, 0};
    CHECK(gdr_op_apply(NULL, s, NULL, NULL, 1, 0) == GDR_ERR_ARG);
    CHECK(gdr_solve(NULL, 1, &s, 1, NULL, NULL, &p, NULL) == GDR_ERR_ARG);
    CHECK(gdr_solve_dr_sh(NULL, 1, &s, NULL, NULL, &p, NULL, NULL) == GDR_ERR_ARG);
    CHECK(gdr_solve_proj_sh(NULL, NULL, 1, &s, 1, NULL, NULL, &p, NULL) == GDR_ERR_ARG);
    CHECK(gdr_defl_export(NULL, NULL, NULL) == GDR_ERR_ARG);
    CHECK(gdr_solve_many(0, NULL, 1, &s, 1, NULL, NULL, &p, NULL) == GDR_ERR_ARG);
    gdr_op none[2] = {NULL, NULL};
    CHECK(gdr_solve_many(2, none, 1, &s, 1, NULL, NULL, &p, NULL) == GDR_ERR_ARG);
    CHECK(p.persistent == 0);
    int dims[4] = {4, 4, 4, 4}, bc[4] = {1, 1, 1, -1};
    gdr_op op = NULL;
    CHECK(gdr_wilson_create(NULL, dims, bc, 0.1, NULL, 0, GDR_LINKS_F32, &op) == GDR_ERR_ARG);
    gdr_op_destroy(NULL);
    gdr_defl_destroy(NULL);
    gdr_ctx_destroy(NULL);

    /* a context: refused without a device, otherwise created and destroyed */
    gdr_ctx c = NULL;
    int rc = gdr_ctx_create(0, NULL, &c);
    if (rc == GDR_OK) {
        CHECK(c != NULL);
        gdr_ctx_destroy(c);
    } else {
        CHECK(c == NULL && rc < 0);
    }

    /* launch-tuning cache */
    CHECK(gdr_tune_load(NULL) == GDR_ERR_ARG);
    snprintf(path, sizeof path, "%s/absent.txt", argv[1]);
    CHECK(gdr_tune_load(path) == GDR_ERR_ARG);
    snprintf(path, sizeof path, "%s/empty.txt", argv[1]);
    write_file(path, "", 0);
    CHECK(gdr_tune_load(path) == 0);
    snprintf(path, sizeof path, "%s/mixed.txt", argv[1]);
    const char* mixed =
        "v1 dslash_r12|gfx950|8x8x8x16|3|0 1 12.5\n"
        "v1 a|b|c 9 1\nv1 a|b|c -1 1\nv1 a|b|c 1 nan\nv1 a|b|c 1 -4\n"
        "v2 a|b|c 1 1\nv1\n\n   \nv1 onlykey\nv1 k 1\n"
        "v1 blk_update|gfx950|7962624|1|4|2 3 0.343\n";
    write_file(path, mixed, strlen(mixed));
    CHECK(gdr_tune_load(path) == 2);
    /* a 6000-character key, a line longer than the reader's buffer */
    snprintf(path, sizeof path, "%s/long.txt", argv[1]);
    {
        size_t n = 6000 + 64;
        char* big = (char*)malloc(n);
        memcpy(big, "v1 ", 3);
        memset(big + 3, 'k', 6000);
        memcpy(big + 6003, " 1 2.0\nv1 x|y|z 2 3.5\n", 22);
        write_file(path, big, 6003 + 22);
        free(big);
    }
    CHECK(gdr_tune_load(path) >= 1);
    /* binary garbage with NULs and no newline at the end */
    snprintf(path, sizeof path, "%s/binary.txt", argv[1]);
    {
        unsigned char junk[3000];
        for (int i = 0; i < 3000; ++i) junk[i] = (unsigned char)((i * 131 + 7) & 0xff);
        write_file(path, (const char*)junk, sizeof junk);
    }
    CHECK(gdr_tune_load(path) >= 0);

    /* report: nothing decided without launches; truncation never overruns */
    CHECK(gdr_tune_report(NULL, 0) == 0);
    char small[3] = {'x', 'x', 'x'};
    CHECK(gdr_tune_report(small, 1) == 0 && small[0] == 0 && small[1] == 'x');
    CHECK(gdr_tune_report(small, 3) == 0 && small[0] == 0);

    if (fails) fprintf(stderr, "%d checks failed\n", fails);
    else printf("asan driver: all checks passed\n");
    return fails ? 1 : 0;
}
