/*
 * Sanitizer driver for the host side of libnsga3 (test infrastructure): the
 * library's sources are compiled for the host only with AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_sanitize.py) and linked with this
 * driver, which calls only what runs without a device: the version and status
 * strings, the workspace-size arithmetic (over the whole range of sizes, where
 * it must never overflow and must grow with N, M and H), and every entry point
 * with arguments that its checks reject before any HIP call.
 */
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "nsga3.h"

static int fails = 0;
#define CHECK(c) do { if (!(c)) { fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); ++fails; } } while (0)

int main(void)
{
    CHECK(nsga3_version() > 0);
    const nsga3_status codes[] = {NSGA3_OK, NSGA3_E_INVALID, NSGA3_E_NONFINITE, NSGA3_E_NOMEM,
                                  NSGA3_E_HIP, NSGA3_E_UNSUPPORTED, (nsga3_status)-99};
    for (size_t q = 0; q < sizeof(codes) / sizeof(codes[0]); ++q) {
        const char *s = nsga3_status_string(codes[q]);
        CHECK(s != NULL && strlen(s) > 0);
    }

    /* workspace sizes: rejected sizes, then monotone growth over the range */
    size_t b = 0;
    CHECK(nsga3_workspace_size(100, 3, 91, NULL) == NSGA3_E_INVALID);
    CHECK(nsga3_workspace_size(0, 3, 91, &b) == NSGA3_E_INVALID);
    CHECK(nsga3_workspace_size(100, 1, 91, &b) == NSGA3_E_INVALID);
    CHECK(nsga3_workspace_size(100, 17, 91, &b) == NSGA3_E_INVALID);
    CHECK(nsga3_workspace_size(100, 3, 0, &b) == NSGA3_E_INVALID);
    CHECK(nsga3_workspace_size(100, 3, 65536, &b) == NSGA3_E_INVALID);
    CHECK(nsga3_workspace_size(2147483648LL, 3, 91, &b) == NSGA3_E_INVALID);
    const int64_t Ns[] = {1, 2, 63, 64, 65, 511, 512, 513, 2047, 2048, 20000, 200000, 1 << 20,
                          1 << 24, 2147483647LL};
    const int32_t Ms[] = {2, 3, 4, 5, 8, 10, 16};
    const int32_t Hs[] = {1, 91, 2048, 4097, 65535};
    size_t prevN = 0;
    for (size_t a = 0; a < sizeof(Ns) / sizeof(Ns[0]); ++a) {
        size_t prevM = 0;
        for (size_t m = 0; m < sizeof(Ms) / sizeof(Ms[0]); ++m) {
            size_t prevH = 0;
            for (size_t h = 0; h < sizeof(Hs) / sizeof(Hs[0]); ++h) {
                size_t w = 0;
                CHECK(nsga3_workspace_size(Ns[a], Ms[m], Hs[h], &w) == NSGA3_OK);
                CHECK(w >= prevH);
                CHECK(w >= (size_t)Ns[a] * 4u * (size_t)Ms[m]);  /* holds at least the records */
                prevH = w;
            }
            CHECK(prevH >= prevM);
            prevM = prevH;
        }
        CHECK(prevM >= prevN);
        prevN = prevM;
    }

    /* entry points with arguments their checks reject before touching HIP */
    nsga3_ctx *ctx = NULL;
    CHECK(nsga3_create(NULL, 0, NULL) == NSGA3_E_INVALID);
    nsga3_destroy(NULL);
    CHECK(nsga3_reserve(NULL, 100, 3, 91) == NSGA3_E_INVALID);
    float f = 0.0f;
    int32_t i32 = 0;
    CHECK(nsga3_select(NULL, &f, 10, 3, &f, 4, 5, &i32, NULL, NULL, NULL, NULL, NULL, NULL, NULL) ==
          NSGA3_E_INVALID);
    CHECK(nsga3_select_noalloc(NULL, 10, 3, &f, 4, 5, &i32, NULL, NULL, NULL, NULL, NULL, NULL,
                               NULL) == NSGA3_E_INVALID);
    CHECK(nsga3_select_noalloc(&f, 10, 3, &f, 4, 11, &i32, NULL, NULL, NULL, NULL, NULL, NULL,
                               NULL) == NSGA3_E_INVALID);                      /* K > N */
    CHECK(nsga3_select_noalloc(&f, 10, 17, &f, 4, 5, &i32, NULL, NULL, NULL, NULL, NULL, NULL,
                               NULL) == NSGA3_E_INVALID);                      /* M > 16 */
    CHECK(nsga3_sbx_pm(NULL, 4, 2, &f, &f, 15.0, 20.0, &f, &f, &f, &i32, NULL) == NSGA3_E_INVALID);
    CHECK(nsga3_sbx_pm(&f, 1, 2, &f, &f, 15.0, 20.0, &f, &f, &f, &i32, NULL) == NSGA3_E_INVALID);
    CHECK(nsga3_sbx_pm(&f, 4, 2, &f, &f, -1.0, 20.0, &f, &f, &f, &i32, NULL) == NSGA3_E_INVALID);
    CHECK(nsga3_gather_rows(NULL, 4, 2, &i32, 1, &f, &i32, NULL) == NSGA3_E_INVALID);
    CHECK(nsga3_gather_rows(&f, 4, 0, &i32, 1, &f, &i32, NULL) == NSGA3_E_INVALID);
    CHECK(nsga3_rvea_select(NULL, &f, 10, 3, &f, 4, 1, 10, 2.0, &i32, NULL, NULL, NULL, NULL) ==
          NSGA3_E_INVALID);
    CHECK(nsga3_hype_select(NULL, &f, 10, 3, &f, &f, 100, 5, &i32, NULL, NULL, NULL, NULL) ==
          NSGA3_E_INVALID);
    nsga3_plan *plan = NULL;
    CHECK(nsga3_plan_create(NULL, NULL, 1, &plan) == NSGA3_E_INVALID);
    CHECK(nsga3_plan_launch(NULL, NULL) == NSGA3_E_INVALID);
    nsga3_plan_destroy(NULL);
    int32_t cnt = 0;
    CHECK(nsga3_tuned_shapes(NULL, NULL, 0, &cnt) == NSGA3_E_INVALID);
    CHECK(nsga3_tuned_save(NULL, "unused.txt") == NSGA3_E_INVALID);
    CHECK(nsga3_tuned_load(NULL, "unused.txt") == NSGA3_E_INVALID);
    double ms[NSGA3_NUM_PHASES];
    int64_t calls = 0;
    CHECK(nsga3_phase_times(NULL, ms, &calls) == NSGA3_E_INVALID);
    CHECK(nsga3_profile(NULL, 1) == NSGA3_E_INVALID);
    (void)ctx;
    if (fails) { fprintf(stderr, "%d checks failed\n", fails); return 1; }
    printf("host ABI sanitizer driver: ok\n");
    return 0;
}
