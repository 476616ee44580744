/* c_abi_client.c -- a plain C99 client of libimpconv: no Python, no torch.
 * It shows that the boundary is usable from C alone (device memory from the
 * HIP runtime, the descriptor-based plan API, status codes and error text),
 * and the tests run it as a child process.
 *
 *   c_abi_client info
 *       version, status strings and argument validation (no GPU needed)
 *   c_abi_client run KIND DTYPE NDIM M0 M1 M2 N0 N1 N2 BATCH M FLAGS DIR
 *       reads DIR/f.bin, DIR/g.bin (and DIR/e.bin for a ternary plan), raw
 *       interleaved complex values in the plan's input layout; runs
 *       impconv_execute on the default stream; writes DIR/h.bin
 *       ([batch][m] in 1D, [batch][n0][n1](...) in 2D/3D).
 * Exit status 0 on success; otherwise the failing call and the library's
 * error text go to stderr. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define __HIP_PLATFORM_AMD__ 1
#include <hip/hip_runtime_api.h>

#include "impconv.h"

static int fail_st(const char* what, impconv_status st)
{
    fprintf(stderr, "%s: %s (%s)\n", what, impconv_status_string(st), impconv_last_error());
    return 1;
}

static int fail_hip(const char* what, hipError_t e)
{
    fprintf(stderr, "%s: %s\n", what, hipGetErrorString(e));
    return 1;
}

/* whole file into a new host buffer */
static void* read_file(const char* path, size_t* bytes)
{
    FILE* fp = fopen(path, "rb");
    void* p = NULL;
    long n;
    if (!fp) return NULL;
    if (fseek(fp, 0, SEEK_END) == 0 && (n = ftell(fp)) > 0 && fseek(fp, 0, SEEK_SET) == 0) {
        p = malloc((size_t)n);
        if (p && fread(p, 1, (size_t)n, fp) != (size_t)n) {
            free(p);
            p = NULL;
        }
        *bytes = (size_t)n;
    }
    fclose(fp);
    return p;
}

/* host file -> new device buffer */
static int upload(const char* dir, const char* name, void** dev)
{
    char path[4096];
    size_t bytes = 0;
    void* host;
    hipError_t e;
    snprintf(path, sizeof(path), "%s/%s", dir, name);
    host = read_file(path, &bytes);
    if (!host) {
        fprintf(stderr, "cannot read %s\n", path);
        return 1;
    }
    e = hipMalloc(dev, bytes);
    if (e == hipSuccess) e = hipMemcpy(*dev, host, bytes, hipMemcpyHostToDevice);
    free(host);
    return e == hipSuccess ? 0 : fail_hip("upload", e);
}

static int info(void)
{
    impconv_desc d;
    impconv_plan* plan = NULL;
    size_t n = 0;
    int bad = 0;
    printf("version %d\n", impconv_version());
    printf("status 0: %s\n", impconv_status_string(IMPCONV_OK));
    printf("status %d: %s\n", (int)IMPCONV_E_SIZE, impconv_status_string(IMPCONV_E_SIZE));
    /* validation that needs no device: null arguments */
    bad |= impconv_plan_create(NULL, NULL) != IMPCONV_E_ARG;
    bad |= impconv_workspace_bytes(NULL, &n) != IMPCONV_E_ARG;
    bad |= impconv_execute(NULL, NULL, NULL, NULL, NULL, NULL, 0, NULL) != IMPCONV_E_ARG;
    bad |= impconv_plan_destroy(NULL) != IMPCONV_OK;
    bad |= impconv_ragged_plan_autotune(NULL, NULL) != IMPCONV_E_ARG;
    memset(&d, 0, sizeof(d));
    d.kind = IMPCONV_COMPLEX;
    d.dtype = 7; /* not a dtype */
    d.ndim = 1;
    d.m[0] = 16;
    d.batch = 1;
    d.M = 1;
    bad |= impconv_plan_create(&plan, &d) != IMPCONV_E_ARG || plan != NULL;
    printf("last error: %s\n", impconv_last_error());
    printf(bad ? "validation FAILED\n" : "validation ok\n");
    return bad;
}

int main(int argc, char** argv)
{
    impconv_desc d;
    impconv_plan* plan = NULL;
    impconv_status st;
    hipError_t e;
    void *f = NULL, *g = NULL, *x = NULL, *h = NULL, *w = NULL, *host = NULL;
    size_t work = 0, cs, out_n, i;
    const char* dir;
    char path[4096];
    FILE* fp;
    int rc = 1;

    if (argc == 2 && strcmp(argv[1], "info") == 0) return info();
    if (argc != 15 || strcmp(argv[1], "run") != 0) {
        fprintf(stderr, "usage: %s info | run KIND DTYPE NDIM M0 M1 M2 N0 N1 N2 BATCH M FLAGS DIR\n", argv[0]);
        return 2;
    }
    memset(&d, 0, sizeof(d));
    d.kind = atoi(argv[2]);
    d.dtype = atoi(argv[3]);
    d.ndim = atoi(argv[4]);
    for (i = 0; i < 3; ++i) {
        d.m[i] = strtoll(argv[5 + i], NULL, 10);
        d.n[i] = strtoll(argv[8 + i], NULL, 10);
    }
    d.batch = strtoll(argv[11], NULL, 10);
    d.M = strtoll(argv[12], NULL, 10);
    d.flags = (uint32_t)strtoul(argv[13], NULL, 10);
    dir = argv[14];
    cs = d.dtype == IMPCONV_C128 ? 16 : 8;

    st = impconv_plan_create(&plan, &d);
    if (st != IMPCONV_OK) return fail_st("impconv_plan_create", st);
    st = impconv_workspace_bytes(plan, &work);
    if (st != IMPCONV_OK) {
        rc = fail_st("impconv_workspace_bytes", st);
        goto done;
    }
    out_n = (size_t)d.batch;
    if (d.ndim == 1) {
        out_n *= (size_t)d.m[0];
    } else {
        for (i = 0; i < (size_t)d.ndim; ++i) out_n *= (size_t)d.n[i];
    }
    if (upload(dir, "f.bin", &f) || upload(dir, "g.bin", &g) ||
        (d.kind == IMPCONV_TERNARY && upload(dir, "e.bin", &x)))
        goto done;
    if ((e = hipMalloc(&h, out_n * cs + 1)) != hipSuccess) {
        rc = fail_hip("hipMalloc h", e);
        goto done;
    }
    if (work && (e = hipMalloc(&w, work)) != hipSuccess) {
        rc = fail_hip("hipMalloc work", e);
        goto done;
    }
    st = impconv_execute(plan, f, g, x, h, w, work, NULL);
    if (st != IMPCONV_OK) {
        rc = fail_st("impconv_execute", st);
        goto done;
    }
    if ((e = hipDeviceSynchronize()) != hipSuccess) {
        rc = fail_hip("hipDeviceSynchronize", e);
        goto done;
    }
    host = malloc(out_n * cs + 1);
    if (!host || (e = hipMemcpy(host, h, out_n * cs, hipMemcpyDeviceToHost)) != hipSuccess) {
        rc = host ? fail_hip("download", e) : 1;
        goto done;
    }
    snprintf(path, sizeof(path), "%s/h.bin", dir);
    fp = fopen(path, "wb");
    if (!fp || fwrite(host, cs, out_n, fp) != out_n) {
        fprintf(stderr, "cannot write %s\n", path);
        if (fp) fclose(fp);
        goto done;
    }
    fclose(fp);
    printf("ok: %zu outputs, workspace %zu bytes\n", out_n, work);
    rc = 0;
done:
    free(host);
    if (f) (void)hipFree(f);
    if (g) (void)hipFree(g);
    if (x) (void)hipFree(x);
    if (h) (void)hipFree(h);
    if (w) (void)hipFree(w);
    (void)impconv_plan_destroy(plan);
    return rc;
}
