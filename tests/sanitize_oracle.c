/* Driver for running the CPU oracle under AddressSanitizer and
 * UndefinedBehaviorSanitizer (test infrastructure; compiled together with
 * oracle/oracle.c by tests/test_sanitizers.py, never part of the product).
 *
 * Exercises every exported routine once at the toy parameters: the Philox
 * known-answer vectors (argv[1] = tests/golden/philox4x32_10_kat.txt), key
 * generation, encryption, the ten gates over all four input rows bootstrapped
 * with extraction and key switching (decryptions checked against the truth
 * tables), the batch blind rotation, extraction, key switching, phases, the
 * negacyclic product against a direct double loop on N = 8, rotation, the
 * modulus switch, the decomposition and the Gaussian sampler. Returns the
 * number of failed checks; the sanitizers abort on the first memory or
 * undefined-behaviour error.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t n, N, k, l, bgbit, t, basebit, pad;
    double sigma_lwe, sigma_ks, sigma_bk;
} or_params;

void or_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]);
int64_t or_gauss_from_block(const uint32_t w[4], double sigma);
void or_negacyclic_mul(int32_t N, const uint32_t *P, const uint32_t *Q, uint32_t *out);
void or_rotate(int32_t N, int32_t a, const uint32_t *P, uint32_t *out);
int32_t or_modswitch(uint32_t x, int32_t two_n);
void or_decompose(uint32_t x, int32_t l, int32_t bgbit, int32_t *digits);
void or_keygen(const or_params *p, uint64_t seed, int32_t *lwe_key, int32_t *tlwe_key, uint32_t *bk, uint32_t *ksk);
void or_encrypt_bits(const or_params *p, const int32_t *lwe_key, uint64_t seed, uint64_t first_index,
                     const uint8_t *bits, int64_t count, uint32_t *out);
uint32_t or_lwe_phase(int32_t dim, const int32_t *key, const uint32_t *ct);
void or_decrypt_bits(int32_t dim, const int32_t *key, const uint32_t *ct, int64_t count, uint8_t *bits);
void or_tlwe_phase(int32_t N, const int32_t *tlwe_key, const uint32_t *acc, uint32_t *phase);
int32_t or_gate_lincomb(int32_t dim, int32_t op, const uint32_t *c1, const uint32_t *c2, uint32_t *out);
void or_blind_rotate(const or_params *p, const uint32_t *bk, const int32_t *bar, uint32_t *acc_out);
void or_sample_extract(int32_t N, const uint32_t *acc, uint32_t *out);
void or_key_switch(const or_params *p, const uint32_t *ksk, const uint32_t *in, uint32_t *out);
int32_t or_bootstrap_batch(const or_params *p, const uint32_t *bk, const uint32_t *ksk, const int32_t *ops,
                           const uint32_t *c1s, const uint32_t *c2s, int64_t count, uint32_t *extracted,
                           uint32_t *outs);
void or_blind_rotate_batch(const or_params *p, const uint32_t *bk, const int32_t *bars, int64_t count,
                           uint32_t *accs);
void or_key_switch_batch(const or_params *p, const uint32_t *ksk, const uint32_t *ins, int64_t count,
                         uint32_t *outs);
void or_modswitch_array(const uint32_t *x, int64_t count, int32_t two_n, int32_t *out);
void or_decompose_array(const uint32_t *x, int64_t count, int32_t l, int32_t bgbit, int32_t *digits);
void or_gauss_array(uint64_t seed, int64_t count, double sigma, int64_t *out);
int32_t or_num_threads(void);

static int failures = 0;

static void check(int ok, const char *what)
{
    if (!ok) {
        fprintf(stderr, "FAILED: %s\n", what);
        failures++;
    }
}

static void *xcalloc(size_t n, size_t size)
{
    void *p = calloc(n, size);
    if (!p) {
        fprintf(stderr, "out of memory\n");
        exit(2);
    }
    return p;
}

/* truth tables in op order, outputs for (a, b) = (0,0), (0,1), (1,0), (1,1) */
static const int kTruth[10][4] = {{1, 1, 1, 0}, {0, 0, 0, 1}, {0, 1, 1, 1}, {0, 1, 1, 0}, {1, 0, 0, 1},
                                  {1, 0, 0, 0}, {0, 1, 0, 0}, {0, 0, 1, 0}, {1, 1, 0, 1}, {1, 0, 1, 1}};

int main(int argc, char **argv)
{
    /* Philox known answers: lines "ctr0 ctr1 ctr2 ctr3 key0 key1 out0 out1 out2 out3" */
    if (argc > 1) {
        FILE *f = fopen(argv[1], "r");
        check(f != NULL, "open known-answer file");
        char line[512];
        int rows = 0;
        while (f && fgets(line, sizeof line, f)) {
            if (line[0] == '#' || line[0] == '\n') continue;
            unsigned v[10];
            if (sscanf(line, "%x %x %x %x %x %x %x %x %x %x", &v[0], &v[1], &v[2], &v[3], &v[4], &v[5], &v[6],
                       &v[7], &v[8], &v[9]) != 10)
                continue;
            const uint32_t ctr[4] = {v[0], v[1], v[2], v[3]}, key[2] = {v[4], v[5]};
            uint32_t out[4];
            or_philox4x32_10(ctr, key, out);
            check(out[0] == v[6] && out[1] == v[7] && out[2] == v[8] && out[3] == v[9], "philox known answer");
            rows++;
        }
        if (f) fclose(f);
        check(rows == 3, "three known-answer rows");
    }

    const or_params p = {256, 512, 1, 3, 7, 8, 2, 0, 1.0 / 32768, 1.0 / 32768, 1.0 / 33554432};
    const int32_t n = p.n, N = p.N, n1 = n + 1, N1 = N + 1;
    const size_t bk_words = (size_t)n * 2 * p.l * 2 * N, ksk_words = (size_t)N * p.t * 4 * n1;
    int32_t *lwe = xcalloc((size_t)n, sizeof *lwe), *tlwe = xcalloc((size_t)N, sizeof *tlwe);
    uint32_t *bk = xcalloc(bk_words, sizeof *bk), *ksk = xcalloc(ksk_words, sizeof *ksk);
    or_keygen(&p, 2021, lwe, tlwe, bk, ksk);

    /* ten gates x four rows */
    const int B = 40;
    uint8_t a[40], b[40], dec[40];
    int32_t ops[40];
    for (int g = 0; g < B; g++) {
        ops[g] = g / 4;
        a[g] = (uint8_t)(g & 1);
        b[g] = (uint8_t)((g >> 1) & 1);
    }
    uint32_t *c1 = xcalloc((size_t)B * n1, sizeof *c1), *c2 = xcalloc((size_t)B * n1, sizeof *c2);
    or_encrypt_bits(&p, lwe, 7, 0, a, B, c1);
    or_encrypt_bits(&p, lwe, 7, B, b, B, c2);
    or_decrypt_bits(n, lwe, c1, B, dec);
    check(memcmp(dec, a, B) == 0, "fresh encryptions decrypt");
    uint32_t *ext = xcalloc((size_t)B * N1, sizeof *ext), *out = xcalloc((size_t)B * n1, sizeof *out);
    check(or_bootstrap_batch(&p, bk, ksk, ops, c1, c2, B, ext, out) == 0, "bootstrap batch");
    or_decrypt_bits(n, lwe, out, B, dec);
    int ok = 1;
    for (int g = 0; g < B; g++) ok &= dec[g] == kTruth[ops[g]][2 * a[g] + b[g]];
    check(ok, "ten gates decrypt to their truth tables");
    or_decrypt_bits(N, tlwe, ext, B, dec);
    ok = 1;
    for (int g = 0; g < B; g++) ok &= dec[g] == kTruth[ops[g]][2 * a[g] + b[g]];
    check(ok, "extracted samples decrypt under the TRLWE key");
    const int32_t bad_op = 10;
    check(or_bootstrap_batch(&p, bk, ksk, &bad_op, c1, c2, 1, NULL, out) != 0, "unknown op refused");

    /* pieces: lincomb, modulus switch, blind rotation, extraction, key switch */
    uint32_t *lin = xcalloc((size_t)n1, sizeof *lin);
    int32_t *bar = xcalloc((size_t)n1, sizeof *bar);
    uint32_t *acc = xcalloc((size_t)2 * N, sizeof *acc), *acc2 = xcalloc((size_t)2 * N, sizeof *acc2);
    uint32_t *e1 = xcalloc((size_t)N1, sizeof *e1), *o1 = xcalloc((size_t)n1, sizeof *o1);
    check(or_gate_lincomb(n, ops[5], c1 + 5 * n1, c2 + 5 * n1, lin) == 0, "lincomb");
    for (int u = 0; u <= n; u++) bar[u] = or_modswitch(lin[u], 2 * N);
    or_blind_rotate(&p, bk, bar, acc);
    or_blind_rotate_batch(&p, bk, bar, 1, acc2);
    check(memcmp(acc, acc2, (size_t)2 * N * sizeof *acc) == 0, "batch blind rotation");
    or_sample_extract(N, acc, e1);
    check(memcmp(e1, ext + 5 * N1, (size_t)N1 * sizeof *e1) == 0, "extraction");
    or_key_switch(&p, ksk, e1, o1);
    check(memcmp(o1, out + 5 * n1, (size_t)n1 * sizeof *o1) == 0, "key switch");
    uint32_t *o2 = xcalloc((size_t)2 * n1, sizeof *o2);
    or_key_switch_batch(&p, ksk, ext, 2, o2);
    check(memcmp(o2, out, (size_t)2 * n1 * sizeof *o2) == 0, "key switch batch");
    uint32_t *ph = xcalloc((size_t)N, sizeof *ph);
    or_tlwe_phase(N, tlwe, acc, ph);
    check(ph[0] == or_lwe_phase(N, tlwe, e1), "phase of the extracted coefficient");

    /* negacyclic product on N = 8 against a direct double loop, and rotation */
    {
        uint32_t P[8], Q[8], R[8], want[8], rot[8];
        for (int i = 0; i < 8; i++) {
            P[i] = (uint32_t)(0x9E3779B9u * (uint32_t)(i + 1));
            Q[i] = (uint32_t)(0x85EBCA6Bu * (uint32_t)(i + 3));
        }
        for (int m = 0; m < 8; m++) {
            uint32_t s = 0;
            for (int i = 0; i < 8; i++)
                for (int j = 0; j < 8; j++) {
                    if (i + j == m) s += P[i] * Q[j];
                    if (i + j == m + 8) s -= P[i] * Q[j];
                }
            want[m] = s;
        }
        or_negacyclic_mul(8, P, Q, R);
        check(memcmp(R, want, sizeof R) == 0, "negacyclic product N = 8");
        or_rotate(8, 11, P, rot);   /* X^11 = -X^3 */
        ok = 1;
        for (int m = 0; m < 8; m++) ok &= rot[m] == (m >= 3 ? 0u - P[m - 3] : P[m + 5]);
        check(ok, "rotation by X^11");
    }

    /* arrays */
    {
        enum { C = 4096 };
        uint32_t *x = xcalloc(C, sizeof *x);
        int32_t *ms = xcalloc(C, sizeof *ms), *dg = xcalloc((size_t)3 * C, sizeof *dg);
        int64_t *gs = xcalloc(C, sizeof *gs);
        for (int i = 0; i < C; i++) x[i] = (uint32_t)i * 1048573u;
        or_modswitch_array(x, C, 1024, ms);
        or_decompose_array(x, C, 3, 7, dg);
        ok = 1;
        for (int i = 0; i < C; i++) {
            int32_t d[3];
            or_decompose(x[i], 3, 7, d);
            ok &= ms[i] == or_modswitch(x[i], 1024) && d[0] == dg[3 * i] && d[1] == dg[3 * i + 1] &&
                  d[2] == dg[3 * i + 2];
        }
        check(ok, "array forms of the modulus switch and decomposition");
        or_gauss_array(5, C, 1.0 / 32768, gs);
        const uint32_t w[4] = {1u, 2u, 3u, 4u};
        (void)or_gauss_from_block(w, 1.0 / 32768);
        free(x); free(ms); free(dg); free(gs);
    }
    check(or_num_threads() >= 1, "thread count");

    free(lwe); free(tlwe); free(bk); free(ksk); free(c1); free(c2); free(ext); free(out);
    free(lin); free(bar); free(acc); free(acc2); free(e1); free(o1); free(o2); free(ph);
    printf("sanitized oracle run: %d failed checks\n", failures);
    return failures;
}
