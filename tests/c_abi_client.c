/* A plain C client of libcemu (test infrastructure): everything through the
 * C ABI of include/cemu.h, device memory from the HIP runtime's C API, no
 * Python and no C++. Built with gcc by tests/test_c_abi.py.
 *
 *   c_abi_client            argument checks only (no GPU needed)
 *   c_abi_client gpu OUT    toy keys from seed 7, 40 gates (every gate op on
 *                           all four input rows) encrypted with seed 11 and
 *                           bootstrapped in both product forms; writes the
 *                           int8 outputs, raw, to the file OUT and checks
 *                           that both forms decrypt to the truth tables.
 * Exit status 0 on success.
 */
#define __HIP_PLATFORM_AMD__ 1
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../include/cemu.h"

static int failures = 0;

static void check(int ok, const char *what)
{
    if (!ok) {
        fprintf(stderr, "FAILED: %s (%s)\n", what, cemu_last_error());
        failures++;
    }
}

static const int kTruth[10][4] = {{1, 1, 1, 0}, {0, 0, 0, 1}, {0, 1, 1, 1}, {0, 1, 1, 0}, {1, 0, 0, 1},
                                  {1, 0, 0, 0}, {0, 1, 0, 0}, {0, 0, 1, 0}, {1, 1, 0, 1}, {1, 0, 1, 1}};

static int argument_checks(void)
{
    cemu_params p;
    check(cemu_params_default(&p, CEMU_STD) == CEMU_OK && p.n == 630 && p.N == 1024, "standard parameters");
    check(cemu_params_default(NULL, CEMU_STD) == CEMU_ERR_NULL, "NULL parameters");
    cemu_secret_key *sk = NULL;
    cemu_cloud_key *ck = NULL;
    p.l = 4;
    check(cemu_keygen(&p, 1, &sk, &ck) == CEMU_ERR_UNSUPPORTED && !sk && !ck, "unsupported gadget refused");
    check(cemu_bootstrap_gates(NULL, 0, NULL, NULL, NULL, NULL, NULL, NULL, 4, NULL) == CEMU_ERR_NULL,
          "NULL cloud key refused");
    check(cemu_lwe_not(630, NULL, NULL, NULL, NULL, -1, NULL) == CEMU_ERR_RANGE, "negative count refused");
    check(strncmp(cemu_version(), "cemu", 4) == 0, "version string");
    return failures;
}

static int gpu_run(const char *out_path)
{
    cemu_params p;
    cemu_secret_key *sk = NULL;
    cemu_cloud_key *ck = NULL;
    check(cemu_params_default(&p, CEMU_TOY) == CEMU_OK, "toy parameters");
    check(cemu_keygen(&p, 7, &sk, &ck) == CEMU_OK, "keygen");
    if (failures) return failures;
    enum { B = 40 };
    const int n1 = p.n + 1;
    uint8_t ops[B], a[B], b[B], bits[B];
    for (int g = 0; g < B; g++) {
        ops[g] = (uint8_t)(g / 4);
        a[g] = (uint8_t)(g & 1);
        b[g] = (uint8_t)((g >> 1) & 1);
    }
    uint32_t *pool = calloc((size_t)2 * B * n1, sizeof *pool);
    uint32_t *out = calloc((size_t)B * n1, sizeof *out);
    int32_t rows[2 * B];
    for (int i = 0; i < 2 * B; i++) rows[i] = i;
    check(pool && out, "host buffers");
    if (failures) return failures;
    check(cemu_encrypt(sk, a, B, 11, 0, pool) == CEMU_OK, "encrypt a");
    check(cemu_encrypt(sk, b, B, 11, B, pool + (size_t)B * n1) == CEMU_OK, "encrypt b");

    uint8_t *d_ops = NULL;
    uint32_t *d_pool = NULL, *d_out = NULL;
    int32_t *d_rows = NULL;
    check(hipMalloc((void **)&d_ops, B) == hipSuccess, "hipMalloc ops");
    check(hipMalloc((void **)&d_pool, sizeof(uint32_t) * 2 * B * n1) == hipSuccess, "hipMalloc pool");
    check(hipMalloc((void **)&d_out, sizeof(uint32_t) * B * n1) == hipSuccess, "hipMalloc out");
    check(hipMalloc((void **)&d_rows, sizeof rows) == hipSuccess, "hipMalloc rows");
    if (failures) return failures;
    check(hipMemcpy(d_ops, ops, B, hipMemcpyHostToDevice) == hipSuccess, "copy ops");
    check(hipMemcpy(d_pool, pool, sizeof(uint32_t) * 2 * B * n1, hipMemcpyHostToDevice) == hipSuccess, "copy pool");
    check(hipMemcpy(d_rows, rows, sizeof rows, hipMemcpyHostToDevice) == hipSuccess, "copy rows");

    const int forms[2] = {CEMU_FORM_INT8, CEMU_FORM_FFT64};
    for (int f = 0; f < 2; f++) {
        const int rc = cemu_bootstrap_gates(ck, forms[f], d_ops, d_pool, d_rows, d_rows + B, NULL, d_out, B, NULL);
        if (forms[f] == CEMU_FORM_FFT64 && p.N != 1024) {
            check(rc == CEMU_ERR_UNSUPPORTED, "FFT64 form refused for N != 1024");
            continue;
        }
        check(rc == CEMU_OK, "bootstrap_gates");
        check(hipDeviceSynchronize() == hipSuccess, "synchronize");
        check(hipMemcpy(out, d_out, sizeof(uint32_t) * B * n1, hipMemcpyDeviceToHost) == hipSuccess, "copy out");
        check(cemu_decrypt(sk, out, B, bits) == CEMU_OK, "decrypt");
        int ok = 1;
        for (int g = 0; g < B; g++) ok &= bits[g] == kTruth[ops[g]][2 * a[g] + b[g]];
        check(ok, "decryptions equal the truth tables");
        if (forms[f] == CEMU_FORM_INT8) {
            FILE *fo = fopen(out_path, "wb");
            check(fo != NULL && fwrite(out, sizeof(uint32_t), (size_t)B * n1, fo) == (size_t)B * n1, "write outputs");
            if (fo) fclose(fo);
        }
    }
    hipFree(d_ops);
    hipFree(d_pool);
    hipFree(d_out);
    hipFree(d_rows);
    free(pool);
    free(out);
    cemu_free_secret_key(sk);
    cemu_free_cloud_key(ck);
    return failures;
}

int main(int argc, char **argv)
{
    if (argc > 2 && strcmp(argv[1], "gpu") == 0) gpu_run(argv[2]);
    else argument_checks();
    printf("c client: %d failed checks\n", failures);
    return failures ? 1 : 0;
}
