/* Host-side argument validation of the C ABI, without a GPU, for a build of
 * the library whose host code carries the address and undefined-behaviour
 * sanitizers (tests/test_host_sanitizers.py builds both and runs this).
 * Every call here must return its documented status without touching a
 * device; a sanitizer report or a wrong status fails the run. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "pfbspec.h"

static int failures = 0;

#define EXPECT(cond)                                                        \
    do {                                                                    \
        if (!(cond)) {                                                      \
            fprintf(stderr, "FAILED line %d: %s (%s)\n", __LINE__, #cond,   \
                    pfbs_last_error());                                     \
            ++failures;                                                     \
        }                                                                   \
    } while (0)

static pfbs_plan_desc desc(int64_t N, int32_t P) {
    pfbs_plan_desc d;
    memset(&d, 0, sizeof d);
    d.N = N;
    d.P = P;
    d.n_pol = 2;
    d.n_int = 4;
    d.device = -1;
    return d;
}

int main(void) {
    pfbs_plan *p = NULL;
    pfbs_batch *b = NULL;
    pfbs_hstream *h = NULL;
    int64_t n = 0;
    EXPECT(pfbs_version() != NULL && strncmp(pfbs_version(), "pfbspec ", 8) == 0);

    /* plan descriptions rejected before any HIP call */
    EXPECT(pfbs_plan_create(&p, 1000, 8, 0, 0, 2, 4) == PFBS_ERR_INVALID && p == NULL);
    EXPECT(strlen(pfbs_last_error()) > 0);
    EXPECT(pfbs_plan_create(&p, 1024, 0, 0, 0, 2, 4) == PFBS_ERR_INVALID);
    EXPECT(pfbs_plan_create(&p, 1024, 8, 0, PFBS_MODE_DIRECT, 2, 4) == PFBS_ERR_INVALID);
    EXPECT(pfbs_plan_create(&p, 1024, 8, 0, 0, 3, 4) == PFBS_ERR_INVALID);
    EXPECT(pfbs_plan_create(&p, 1024, 8, 0, 0, 2, 0) == PFBS_ERR_INVALID);
    EXPECT(pfbs_plan_create(NULL, 1024, 8, 0, 0, 2, 4) == PFBS_ERR_INVALID);
    EXPECT(pfbs_plan_create_ex(&p, NULL) == PFBS_ERR_INVALID);
    pfbs_plan_desc d = desc(1 << 19, 8);
    d.window = PFBS_WINDOW_CUSTOM;   /* custom window without taps */
    EXPECT(pfbs_plan_create_ex(&p, &d) == PFBS_ERR_INVALID);
    d = desc(1 << 15, 8);
    d.split_n2 = 100;
    EXPECT(pfbs_plan_create_ex(&p, &d) == PFBS_ERR_INVALID);
    d = desc(1 << 15, 8);
    d.tap_unroll = 3;
    EXPECT(pfbs_plan_create_ex(&p, &d) == PFBS_ERR_INVALID);
    d = desc(1 << 15, 8);
    d.col_pair = -1;
    EXPECT(pfbs_plan_create_ex(&p, &d) == PFBS_ERR_INVALID);
    d = desc(1024, 8);
    d.n_pol = 1;
    d.output = PFBS_OUT_STOKES;
    EXPECT(pfbs_plan_create_ex(&p, &d) == PFBS_ERR_INVALID);

    /* a valid description with no device: a device or support error, no crash */
    d = desc(1 << 15, 8);
    pfbs_status st = pfbs_plan_create_ex(&p, &d);
    EXPECT(st == PFBS_ERR_DEVICE || st == PFBS_ERR_UNSUPPORTED || st == PFBS_ERR_NOMEM);
    EXPECT(p == NULL);

    /* calls on no plan, or on memory that is not a plan */
    EXPECT(pfbs_plan_destroy(NULL) == PFBS_OK);
    EXPECT(pfbs_dumps_in(NULL, 1024) == -1);
    EXPECT(pfbs_execute(NULL, NULL, 1024, NULL, 0, &n, NULL) == PFBS_ERR_STATE);
    EXPECT(pfbs_execute(NULL, NULL, 1024, NULL, 0, NULL, NULL) == PFBS_ERR_INVALID);
    EXPECT(pfbs_execute_noalloc(NULL, NULL, 1024, NULL, 0, &n, NULL) == PFBS_ERR_STATE);
    EXPECT(pfbs_flush(NULL, NULL, &n, NULL) == PFBS_ERR_STATE);
    EXPECT(pfbs_plan_reset(NULL) == PFBS_ERR_STATE);
    pfbs_plan_info info;
    EXPECT(pfbs_plan_get_info(NULL, &info) == PFBS_ERR_STATE);
    EXPECT(pfbs_debug_table(NULL, 0, NULL, 0, &n, NULL) == PFBS_ERR_STATE);
    EXPECT(pfbs_plan_timing(NULL, 1) == PFBS_ERR_STATE);
    void *fake = calloc(1, 4096);      /* zeroed: no live-plan tag */
    EXPECT(pfbs_plan_destroy((pfbs_plan *)fake) == PFBS_ERR_STATE);
    EXPECT(pfbs_dumps_in((pfbs_plan *)fake, 1024) == -1);
    EXPECT(pfbs_execute((pfbs_plan *)fake, fake, 1024, NULL, 0, &n, NULL) == PFBS_ERR_STATE);
    free(fake);

    /* batches and host streams */
    EXPECT(pfbs_batch_create(&b, NULL, 1) == PFBS_ERR_INVALID);
    d = desc(1000, 8);
    EXPECT(pfbs_batch_create(&b, &d, 1) == PFBS_ERR_INVALID && b == NULL);
    pfbs_plan_desc two[2] = {desc(4096, 8), desc(4096, 8)};
    two[1].n_pol = 1;                  /* mixed polarisation counts */
    EXPECT(pfbs_batch_create(&b, two, 2) == PFBS_ERR_INVALID);
    EXPECT(pfbs_batch_create(&b, two, 0) == PFBS_ERR_INVALID);
    EXPECT(pfbs_batch_destroy(NULL) == PFBS_OK);
    EXPECT(pfbs_batch_plan(NULL, 0) == NULL);
    d = desc(4096, 8);
    EXPECT(pfbs_hstream_create(&h, &d, 4096 * 8, 1) == PFBS_ERR_INVALID);
    EXPECT(pfbs_hstream_create(&h, &d, 4096 * 8 + 1, 2) == PFBS_ERR_INVALID);
    EXPECT(pfbs_hstream_create(&h, NULL, 4096 * 8, 2) == PFBS_ERR_INVALID);
    EXPECT(pfbs_hstream_destroy(NULL) == PFBS_OK);
    EXPECT(pfbs_host_free(NULL) == PFBS_OK);
    EXPECT(pfbs_autotune(NULL, 0, 0, NULL, NULL) == PFBS_ERR_INVALID);

    if (failures) {
        fprintf(stderr, "%d check(s) failed\n", failures);
        return 1;
    }
    printf("host validation ok\n");
    return 0;
}
