/* Host-only use of the C ABI from plain C (no Python): plans, multi-template planning, sample
 * sizes and estimates. Built and run by tests/test_c_abi.py; prints one line per check. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "cc.h"

static int fails = 0;
#define CHECK(cond, ...)                    \
    do {                                    \
        if (!(cond)) {                      \
            ++fails;                        \
            printf("FAIL: " __VA_ARGS__);   \
            printf("\n");                   \
        }                                   \
    } while (0)

int main(void) {
    /* the 5-path 0-1-2-3-4 and a spider with two equal legs */
    const int32_t path5[] = {0, 1, 1, 2, 2, 3, 3, 4};
    const int32_t spider[] = {0, 1, 1, 2, 0, 3, 3, 4};
    cc_plan *p = NULL, *q = NULL, *r = NULL;
    CHECK(cc_plan_create(5, path5, -1, 0, &p) == CC_OK, "plan create: %s", cc_last_error());
    CHECK(cc_plan_create(5, spider, 0, 0, &q) == CC_OK, "spider: %s", cc_last_error());
    CHECK(cc_plan_create(5, spider, 0, CC_PLAN_NO_SHARING, &r) == CC_OK, "spider unshared: %s", cc_last_error());
    cc_plan_info ip, iq, ir;
    CHECK(cc_plan_info_get(p, &ip) == CC_OK && ip.k == 5 && ip.aut == 2.0, "path info");
    CHECK(ip.units_per_edge == 22, "path units %lld", (long long)ip.units_per_edge);
    CHECK(cc_plan_info_get(q, &iq) == CC_OK && cc_plan_info_get(r, &ir) == CC_OK, "spider info");
    CHECK(iq.aut == 2.0 && ir.n_splits == 4 && iq.n_splits < ir.n_splits, "spider splits %d %d", iq.n_splits,
          ir.n_splits);
    int32_t s, a, pp;
    CHECK(cc_plan_split_get(p, ip.n_splits - 1, &s, &a, &pp) == CC_OK && s == 5 && a + pp == 5, "root split");

    /* errors come back as status codes with a message, never as aborts */
    const int32_t cycle[] = {0, 1, 1, 2, 2, 0};
    cc_plan* bad = NULL;
    CHECK(cc_plan_create(4, cycle, -1, 0, &bad) == CC_EINVAL && bad == NULL, "cycle rejected");
    CHECK(strlen(cc_last_error()) > 0, "error message");
    CHECK(cc_plan_create(17, path5, -1, 0, &bad) == CC_ERANGE, "k range");

    /* multi-template planning over both templates */
    const cc_plan* both[] = {p, r};
    cc_multi* m = NULL;
    CHECK(cc_multi_create(2, both, &m) == CC_OK, "multi: %s", cc_last_error());
    int32_t steps = 0, tables = 0;
    int64_t splits = 0;
    CHECK(cc_multi_info_get(m, &steps, &splits, &tables) == CC_OK && splits == ip.n_splits + ir.n_splits &&
              steps < splits,
          "multi info %d %lld", steps, (long long)splits);
    int32_t pl, sp;
    CHECK(cc_multi_step_get(m, steps - 1, &pl, &sp) == CC_OK && pl == 1, "last step belongs to the last template");
    CHECK(cc_multi_step_get(m, steps, &pl, &sp) == CC_ERANGE, "step range");
    cc_multi_destroy(m);

    /* sample sizes and estimates */
    int64_t per = 0;
    int32_t groups = 0;
    CHECK(cc_iterations(5, 0.5, 0.1, &per, &groups) == CC_OK, "iterations");
    CHECK(per == (int64_t)ceil(4.0 * exp(5.0) / 0.25) && groups == (int32_t)ceil(8.0 * log(10.0)), "iteration sizes");
    const double X[4] = {10.0, 20.0, 30.0, 40.0};
    double est = 0.0, se = 0.0;
    CHECK(cc_estimate(p, X, 4, &est, &se) == CC_OK, "estimate");
    const double f = pow(5.0, 5.0) / 120.0 / 2.0;
    CHECK(fabs(est - 25.0 * f) <= 1e-12 * est, "estimate value %.17g", est);

    /* the planner's tables read back: offsets inside the constants, root split writes the full template */
    cc_plan_info pi;
    CHECK(cc_plan_info_get(p, &pi) == CC_OK, "plan info");
    unsigned char* consts = (unsigned char*)malloc(pi.device_bytes ? pi.device_bytes : 1);
    CHECK(consts != NULL && cc_plan_constants_get(p, consts, pi.device_bytes) == CC_OK, "constants");
    CHECK(pi.device_bytes == 0 || cc_plan_constants_get(p, consts, pi.device_bytes - 1) == CC_ENOSPC, "constants size");
    for (int32_t i = 0; i < pi.n_splits; ++i) {
        cc_split_maps sm;
        CHECK(cc_plan_split_maps(p, i, &sm) == CC_OK, "split maps %d", i);
        CHECK(sm.split_off >= 0 && (size_t)sm.split_off < pi.device_bytes, "split list offset %d", i);
        CHECK((sm.out == -2) == (i == pi.n_splits - 1), "root split writes the template %d", i);
    }
    CHECK(cc_plan_split_maps(p, pi.n_splits, NULL) == CC_EINVAL, "split maps NULL");
    free(consts);

    /* storage order of table rows: a permutation of colex ranks; short rows keep colex order */
    int32_t order[462];
    int seen[462] = {0};
    CHECK(cc_entry_order(12, 5, order, 462) == CC_OK, "entry order: %s", cc_last_error());
    int perm = 1;
    for (int i = 0; i < 462; ++i) {
        if (order[i] < 0 || order[i] >= 462 || seen[order[i]]) perm = 0;
        else seen[order[i]] = 1;
    }
    CHECK(perm, "entry order is a permutation");
    CHECK(cc_entry_order(12, 1, order, 11) == CC_OK && order[0] == 0 && order[10] == 10, "short rows in colex order");
    CHECK(cc_entry_order(12, 5, order, 461) == CC_EINVAL, "entry order size check");
    CHECK(cc_entry_order(12, 12, order, 1) == CC_ERANGE, "entry order m range");

    cc_plan_destroy(p);
    cc_plan_destroy(q);
    cc_plan_destroy(r);
    printf("%s\n", fails ? "FAILED" : "OK");
    return fails ? 1 : 0;
}
