/* The device entry points of the C ABI from plain C (no C++, no Python): a cycle C_n whose
 * vertex i has colour i mod k, where the number of colourful labelled k-paths is 2n and every
 * tree with a vertex of degree 3 has none (closed forms of Eq. 1's count). Device memory comes
 * from the HIP runtime's C API. Built and run by tests/test_c_abi.py on a GPU; prints one line
 * per failed check and OK at the end. */
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>

#include "cc.h"

static int fails = 0;
#define CHECK(cond, ...)                  \
    do {                                  \
        if (!(cond)) {                    \
            ++fails;                      \
            printf("FAIL: " __VA_ARGS__); \
            printf("\n");                 \
        }                                 \
    } while (0)

static void* dalloc(size_t bytes) {
    void* p = NULL;
    if (hipMalloc(&p, bytes < 256 ? 256 : bytes) != hipSuccess) {
        printf("FAIL: hipMalloc %zu\n", bytes);
        exit(1);
    }
    return p;
}

/* X of the template on the cycle for B copies of the colouring i mod k, plain and packed */
static void count_on_cycle(const cc_graph* g, int64_t n, int32_t k, const int32_t* edges, double want) {
    cc_plan* p = NULL;
    CHECK(cc_plan_create(k, edges, -1, 0, &p) == CC_OK, "plan: %s", cc_last_error());
    cc_plan_info info;
    CHECK(cc_plan_info_get(p, &info) == CC_OK, "plan info");
    void* consts = dalloc(info.device_bytes);
    CHECK(cc_plan_bind_device(p, consts, info.device_bytes, NULL) == CC_OK, "bind: %s", cc_last_error());
    const int32_t B = 2;
    uint8_t* col = (uint8_t*)malloc((size_t)(B * n));
    for (int32_t b = 0; b < B; ++b)
        for (int64_t i = 0; i < n; ++i) col[b * n + i] = (uint8_t)(i % k);
    uint8_t* dcol = (uint8_t*)dalloc((size_t)(B * n));
    CHECK(hipMemcpy(dcol, col, (size_t)(B * n), hipMemcpyHostToDevice) == hipSuccess, "colours upload");
    size_t wsb = 0, wsp = 0;
    CHECK(cc_count_workspace_bytes(p, g, &wsb) == CC_OK, "ws bytes");
    CHECK(cc_count_packed_workspace_bytes(p, g, B, &wsp) == CC_OK, "packed ws bytes");
    void* ws = dalloc(wsb > wsp ? wsb : wsp);
    double* dX = (double*)dalloc(2 * B * sizeof(double));
    CHECK(cc_count(p, g, dcol, B, ws, wsb, dX, NULL, NULL) == CC_OK, "count: %s", cc_last_error());
    CHECK(cc_count_packed(p, g, dcol, B, ws, wsp, dX + B, NULL, NULL) == CC_OK, "packed: %s", cc_last_error());
    CHECK(cc_stream_check(NULL) == CC_OK, "stream: %s", cc_last_error());
    double X[4];
    CHECK(hipMemcpy(X, dX, sizeof X, hipMemcpyDeviceToHost) == hipSuccess, "X download");
    for (int i = 0; i < 2 * B; ++i) CHECK(X[i] == want, "k=%d X[%d] = %.17g, want %.17g", k, i, X[i], want);
    /* a workspace one byte short is refused before any launch */
    CHECK(cc_count(p, g, dcol, B, ws, wsb - 1, dX, NULL, NULL) == CC_ENOSPC, "short workspace");
    (void)hipFree(dX);
    (void)hipFree(ws);
    (void)hipFree(dcol);
    (void)hipFree(consts);
    free(col);
    cc_plan_destroy(p);
}

int main(void) {
    const int64_t n = 600, nnz = 2 * n;
    int64_t* rp = (int64_t*)malloc((size_t)(n + 1) * sizeof(int64_t));
    int32_t* cl = (int32_t*)malloc((size_t)nnz * sizeof(int32_t));
    for (int64_t i = 0; i < n; ++i) {
        int32_t a = (int32_t)((i + n - 1) % n), b = (int32_t)((i + 1) % n);
        rp[i] = 2 * i;
        cl[2 * i] = a < b ? a : b;
        cl[2 * i + 1] = a < b ? b : a;
    }
    rp[n] = nnz;
    int64_t* drp = (int64_t*)dalloc((size_t)(n + 1) * sizeof(int64_t));
    int32_t* dcl = (int32_t*)dalloc((size_t)nnz * sizeof(int32_t));
    CHECK(hipMemcpy(drp, rp, (size_t)(n + 1) * sizeof(int64_t), hipMemcpyHostToDevice) == hipSuccess, "rp");
    CHECK(hipMemcpy(dcl, cl, (size_t)nnz * sizeof(int32_t), hipMemcpyHostToDevice) == hipSuccess, "col");
    size_t gwb = 0;
    CHECK(cc_graph_workspace_bytes(n, nnz, NULL, &gwb) == CC_OK, "graph ws bytes");
    void* gws = dalloc(gwb);
    cc_graph* g = NULL;
    CHECK(cc_graph_prepare(n, nnz, drp, dcl, gws, gwb, NULL, 0, NULL, &g) == CC_OK, "prepare: %s", cc_last_error());
    if (!g) return 1;

    const int32_t path5[] = {0, 1, 1, 2, 2, 3, 3, 4};
    const int32_t path3[] = {0, 1, 1, 2};
    const int32_t star4[] = {0, 1, 0, 2, 0, 3};
    count_on_cycle(g, n, 5, path5, 2.0 * n);
    count_on_cycle(g, n, 3, path3, 2.0 * n);
    count_on_cycle(g, n, 4, star4, 0.0);

    /* the colouring kernel writes colours below k */
    uint8_t* dcol = (uint8_t*)dalloc((size_t)n);
    CHECK(cc_color(g, 7, 99, 0, 1, dcol, NULL) == CC_OK, "color");
    uint8_t* c = (uint8_t*)malloc((size_t)n);
    CHECK(hipMemcpy(c, dcol, (size_t)n, hipMemcpyDeviceToHost) == hipSuccess, "colour download");
    int bad = 0;
    for (int64_t i = 0; i < n; ++i) bad += c[i] >= 7;
    CHECK(bad == 0, "%d colours out of range", bad);

    /* an asymmetric CSR is refused by the device-side validation */
    cl[1] = (int32_t)((cl[1] + 7) % n);
    CHECK(hipMemcpy(dcl, cl, (size_t)nnz * sizeof(int32_t), hipMemcpyHostToDevice) == hipSuccess, "col");
    cc_graph* g2 = NULL;
    CHECK(cc_graph_prepare(n, nnz, drp, dcl, gws, gwb, NULL, 0, NULL, &g2) == CC_EINVAL && g2 == NULL,
          "broken CSR accepted");

    cc_graph_release(g);
    (void)hipFree(dcol);
    (void)hipFree(gws);
    (void)hipFree(dcl);
    (void)hipFree(drp);
    free(c);
    free(rp);
    free(cl);
    printf(fails ? "FAILED %d\n" : "OK\n", fails);
    return fails ? 1 : 0;
}
