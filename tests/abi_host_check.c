/* Host-side exercise of the C ABI (include/qless.h) for the sanitizer build
 * in test_abi_sanitizers.py: every size query over a grid of arguments
 * (extreme ones included), the tuning table, batch plans built and
 * destroyed, and the argument checks of the entry points.  Nothing here
 * reaches a kernel launch, so it runs without a GPU.  Exit status 0 when
 * every expectation holds. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "qless.h"

static int failures = 0;
#define EXPECT(cond)                                                        \
    do {                                                                    \
        if (!(cond)) {                                                      \
            fprintf(stderr, "%s:%d: expectation failed: %s\n", __FILE__, __LINE__, #cond); \
            ++failures;                                                     \
        }                                                                   \
    } while (0)

static double *const FAKE = (double *)(uintptr_t)0x100000; /* never dereferenced on the host */

int main(void) {
    const int64_t ms[] = {-1, 0, 1, 2, 63, 64, 65, 1000, 65537, 1000000, 50000000, (int64_t)1 << 34};
    const int nm = (int)(sizeof ms / sizeof ms[0]);
    for (int s = -12; s <= 2; ++s) EXPECT(qless_status_string(s) != NULL);
    EXPECT(qless_version() != NULL);

    /* size queries */
    for (int method = -1; method <= 8; ++method)
        for (int i = 0; i < nm; ++i)
            for (int64_t n = -1; n <= QLESS_MAX_N + 2; ++n) {
                const size_t b = qless_workspace_bytes(method, ms[i], n);
                if (n < 1 || ms[i] < 0) EXPECT(b == 0);
                (void)b;
            }
    EXPECT(qless_noalloc_scratch_bytes() > 0);
    for (int i = 0; i < nm; ++i)
        for (int64_t p = -1; p <= 65; p += 4)
            for (int64_t n = -1; n <= 65; n += 3) {
                const size_t b = qless_two_phase_workspace_bytes(ms[i], p, n);
                if (p + n > QLESS_MAX_N || n < 1 || p < 0) EXPECT(b == 0);
            }
    for (int i = 0; i < nm; ++i)
        for (int64_t n = -1; n <= 300; n += 37)
            for (int64_t panel = -1; panel <= 80; panel += 27) (void)qless_wide_workspace_bytes(ms[i], n, panel);
    for (int i = 0; i < nm; ++i)
        for (int64_t n = -1; n <= QLESS_MAX_N + 2; ++n) (void)qless_tsqr_state_bytes(ms[i], n);

    /* tuning table */
    for (int64_t n = -1; n <= QLESS_MAX_N + 1; ++n) {
        int32_t w = -1, f = -1, r = -1;
        const int ok = qless_tune_get(n, &w, &f, &r);
        if (n >= 1 && n <= QLESS_MAX_N) {
            EXPECT(ok == QLESS_OK && w > 0 && f >= 2 && r >= 1);
            EXPECT(qless_tune_set(n, 12, 8, 0) == QLESS_OK);
            EXPECT(qless_tune_set(n, 64, 8, 0) != QLESS_OK);
            EXPECT(qless_tune_set(n, 8, 1, 0) != QLESS_OK);
            EXPECT(qless_tune_set(n, 8, 0, 999) != QLESS_OK);
            (void)qless_workspace_bytes(QLESS_METHOD_TSQR, 50000000, n);
            EXPECT(qless_tune_set(n, 0, 0, 0) == QLESS_OK);
        } else {
            EXPECT(ok != QLESS_OK);
        }
    }

    /* batch plans on host descriptors */
    enum { NB = 40 };
    qless_matrix_desc d[NB];
    for (int i = 0; i < NB; ++i) {
        d[i].X = FAKE;
        d[i].m = (int64_t)(i * 7919) % 3000001;
        d[i].n = 1 + (i * 13) % QLESS_MAX_N;
        d[i].ldx = d[i].n;
        d[i].R = FAKE;
        d[i].ldr = d[i].n;
        d[i].accumulate = i & 1;
    }
    for (int count = 0; count <= NB; count += 5)
        for (int64_t tile = -1; tile <= (1 << 22); tile += (1 << 20)) {
            qless_batch_plan *plan = NULL;
            const int st = qless_batch_plan_create(d, count, tile, 0, &plan);
            if (st == QLESS_OK) {
                EXPECT(plan != NULL);
                (void)qless_batch_plan_workspace_bytes(plan);
                EXPECT(qless_batch_plan_tiles(plan) >= 0);
                qless_batch_plan_destroy(plan);
            }
        }
    d[3].n = QLESS_MAX_N + 1;
    {
        qless_batch_plan *plan = NULL;
        EXPECT(qless_batch_plan_create(d, NB, 0, 0, &plan) != QLESS_OK);
    }
    d[3].n = 5;
    d[4].ldx = d[4].n - 1;
    {
        qless_batch_plan *plan = NULL;
        EXPECT(qless_batch_plan_create(d, NB, 0, 0, &plan) != QLESS_OK);
    }

    /* argument checks of the entry points (no launch happens) */
    EXPECT(qless_tsqr_r(FAKE, 100, 0, 4, FAKE, 4, NULL, 0, NULL) == QLESS_ERR_ARG);
    EXPECT(qless_tsqr_r(FAKE, 100, 65, 65, FAKE, 65, NULL, 0, NULL) == QLESS_ERR_UNSUPPORTED);
    EXPECT(qless_tsqr_r(FAKE, 100, 4, 3, FAKE, 4, NULL, 0, NULL) == QLESS_ERR_ARG);
    EXPECT(qless_tsqr_r(FAKE, 50000000, 8, 8, FAKE, 8, NULL, 0, NULL) == QLESS_ERR_WORKSPACE);
    EXPECT(qless_tsqr_r_noalloc(FAKE, (int64_t)1 << 40, 64, 64, FAKE, 64, NULL) != QLESS_OK);
    EXPECT(qless_two_phase_r(FAKE, 4, 1 << 20, FAKE, 10000000, 3, 3, FAKE, 3, FAKE, 3, FAKE, (size_t)1 << 30, NULL) ==
           QLESS_ERR_UNSUPPORTED);
    EXPECT(qless_tsqr_state_init(FAKE, 1, 1000, 4, NULL) != QLESS_OK);
    EXPECT(qless_timing_enable(0) == QLESS_OK);
    EXPECT(qless_timing_reset() == QLESS_OK);
    {
        double ms_total = -1.0;
        int64_t count = -1;
        EXPECT(qless_timing_read("tsqr_stage1", &ms_total, &count) == QLESS_OK && count == 0);
        EXPECT(qless_timing_read("no such kernel", &ms_total, &count) != QLESS_OK);
    }
    if (failures) fprintf(stderr, "%d expectation(s) failed\n", failures);
    return failures ? 1 : 0;
}
