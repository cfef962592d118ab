/* A plain C11 program that uses the library only through include/fsb.h and
 * the HIP runtime's C API: no C++, no Python, no torch.  It shows that the
 * boundary is a C ABI of plain pointers and sizes.
 *
 *   c_consumer host
 *       host-side checks only (no device memory, no kernel): ABI version,
 *       workspace size, rejected arguments.
 *   c_consumer run N STEPS MODE SEED OUT
 *       one school of N fish (the default configuration of the library:
 *       pond half-width 100, swim step 0.1, weights [1, 2) within [1, 4]),
 *       STEPS iterations by fsb_run(MODE), then writes the five float32
 *       columns (x, y, w, prev, cur, N values each) to the file OUT and
 *       prints M and the sums of the last iteration in C99 hex-float.
 */
#define __HIP_PLATFORM_AMD__
#include <hip/hip_runtime_api.h>

#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "fsb.h"

static void need(int ok, const char *what) {
    if (!ok) {
        fprintf(stderr, "c_consumer: %s\n", what);
        exit(1);
    }
}

static void fsb_ok(int rc, const char *what) {
    if (rc != FSB_OK) {
        fprintf(stderr, "c_consumer: %s: %s (%s)\n", what, fsb_strerror(rc), fsb_last_error());
        exit(1);
    }
}

static void hip_ok(hipError_t e, const char *what) {
    if (e != hipSuccess) {
        fprintf(stderr, "c_consumer: %s: %s\n", what, hipGetErrorString(e));
        exit(1);
    }
}

static fsb_config default_config(uint64_t n, uint64_t seed, uint32_t history) {
    fsb_config c;
    memset(&c, 0, sizeof c);
    c.n_fish = n;
    c.seed = seed;
    c.pond_half = 100.0f;
    c.swim_step = 0.1f;
    c.w_init_lo = 1.0f;
    c.w_init_hi = 2.0f;
    c.w_min = 1.0f;
    c.w_max = 4.0f;
    c.reduce_mode = FSB_REDUCE_COMPENSATED;
    c.history_len = history;
    c.swim_rule = 0;
    return c;
}

static int host_checks(void) {
    need(fsb_abi_version() == FSB_ABI_VERSION, "ABI version");
    fsb_config c = default_config(1000, 0, 16);
    size_t bytes = 0;
    fsb_ok(fsb_workspace_bytes(&c, &bytes), "fsb_workspace_bytes");
    need(bytes > 0 && bytes % 256 == 0, "workspace size");
    /* rejected on the host, before any HIP call */
    c.pond_half = 0.0f;
    need(fsb_workspace_bytes(&c, &bytes) == FSB_ERR_INVALID_ARG, "pond_half 0 rejected");
    c = default_config(0, 0, 16);
    fsb_state none;
    memset(&none, 0, sizeof none);
    fsb_school *h = NULL;
    need(fsb_init(&c, none, NULL, 0, NULL, &h) == FSB_ERR_INVALID_ARG && h == NULL,
         "n_fish 0 rejected");
    need(fsb_run(NULL, 1, FSB_RUN_PLAIN) == FSB_ERR_INVALID_ARG, "NULL handle rejected");
    need(strcmp(fsb_strerror(FSB_OK), "ok") == 0, "strerror");
    printf("host ok: workspace %zu bytes for 1000 fish\n", bytes);
    return 0;
}

static int run(uint64_t n, uint32_t steps, uint32_t mode, uint64_t seed, const char *out) {
    fsb_config c = default_config(n, seed, steps > 0 ? steps : 1);
    size_t ws_bytes = 0;
    fsb_ok(fsb_workspace_bytes(&c, &ws_bytes), "fsb_workspace_bytes");
    float *col[5];
    for (int k = 0; k < 5; ++k) hip_ok(hipMalloc((void **)&col[k], n * sizeof(float)), "hipMalloc");
    void *ws = NULL;
    hip_ok(hipMalloc(&ws, ws_bytes), "hipMalloc workspace");
    hipStream_t stream;
    hip_ok(hipStreamCreate(&stream), "hipStreamCreate");
    fsb_state st = {col[0], col[1], col[2], col[3], col[4]};
    fsb_school *h = NULL;
    fsb_ok(fsb_init(&c, st, ws, ws_bytes, (void *)stream, &h), "fsb_init");
    fsb_ok(fsb_run(h, steps, mode), "fsb_run");
    double xy[2], sums[3];
    float M = 0.0f;
    fsb_ok(fsb_barycentre(h, xy, sums), "fsb_barycentre");
    fsb_ok(fsb_max_delta(h, &M), "fsb_max_delta");
    uint64_t t = 0;
    fsb_ok(fsb_step_index(h, &t), "fsb_step_index");
    fsb_ok(fsb_sync(h), "fsb_sync");

    float *host = (float *)malloc(n * sizeof(float));
    need(host != NULL, "malloc");
    FILE *f = fopen(out, "wb");
    need(f != NULL, "cannot open the output file");
    for (int k = 0; k < 5; ++k) {
        hip_ok(hipMemcpy(host, col[k], n * sizeof(float), hipMemcpyDeviceToHost), "hipMemcpy");
        need(fwrite(host, sizeof(float), n, f) == n, "short write");
    }
    fclose(f);
    free(host);
    printf("t %llu\nM %a\nsums %a %a %a\nxy %a %a\n", (unsigned long long)t, (double)M, sums[0],
           sums[1], sums[2], xy[0], xy[1]);

    fsb_ok(fsb_destroy(h), "fsb_destroy");
    hip_ok(hipStreamDestroy(stream), "hipStreamDestroy");
    hip_ok(hipFree(ws), "hipFree");
    for (int k = 0; k < 5; ++k) hip_ok(hipFree(col[k]), "hipFree");
    return 0;
}

int main(int argc, char **argv) {
    if (argc == 2 && strcmp(argv[1], "host") == 0) return host_checks();
    if (argc == 7 && strcmp(argv[1], "run") == 0) {
        const uint64_t n = strtoull(argv[2], NULL, 10);
        const uint32_t steps = (uint32_t)strtoul(argv[3], NULL, 10);
        const uint32_t mode = (uint32_t)strtoul(argv[4], NULL, 10);
        const uint64_t seed = strtoull(argv[5], NULL, 10);
        need(n > 0, "N must be >= 1");
        return run(n, steps, mode, seed, argv[6]);
    }
    fprintf(stderr, "usage: c_consumer host | c_consumer run N STEPS MODE SEED OUT\n");
    return 2;
}
