/* Exhaustive pins of the oracle's modulus switch and gadget decomposition
 * over all 2^32 torus words (test infrastructure; linked with oracle.c).
 *
 * Each property is a characterisation independent of how the oracle computes
 * the value:
 *  - modulus switch to Z/2N: abar in [0, 2N) and x * 2N - abar * 2^32, taken
 *    modulo 2N * 2^32 into [-2N * 2^31, 2N * 2^31), lies in [-2^31, 2^31):
 *    abar is the nearest integer to x * 2N / 2^32 modulo 2N, ties going up;
 *  - decomposition with l = 3, Bgbit = 7: every digit in [-64, 64), the
 *    recomposition sum_j d_j 2^(32 - 7j) is a multiple of 2^11 modulo 2^32,
 *    and x minus it, taken modulo 2^32 into [-2^31, 2^31), lies in
 *    [-2^10, 2^10) (nearest multiple, ties up). A balanced base-128
 *    representation of a multiple of 2^11 is unique, so these fix the digits.
 * Prints the number of violations of each property and exits nonzero if any.
 */
#include <stdint.h>
#include <stdio.h>

int32_t or_modswitch(uint32_t x, int32_t two_n);
void or_decompose(uint32_t x, int32_t l, int32_t bgbit, int32_t *digits);

static int64_t centred(int64_t v, int64_t modulus)
{
    v %= modulus;
    if (v < 0) v += modulus;
    return v >= modulus / 2 ? v - modulus : v;
}

int main(void)
{
    long long bad_ms[2] = {0, 0}, bad_range = 0, bad_mult = 0, bad_err = 0;
    const int32_t two_ns[2] = {1024, 2048};
    for (int k = 0; k < 2; k++) {
        const int64_t tn = two_ns[k];
        long long bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : bad)
        for (int64_t i = 0; i < (1LL << 32); i++) {
            const int32_t a = or_modswitch((uint32_t)i, (int32_t)tn);
            const int64_t d = centred(i * tn - (int64_t)a * (1LL << 32), tn << 32);
            if (a < 0 || a >= tn || d < -(1LL << 31) || d >= (1LL << 31)) bad++;
        }
        bad_ms[k] = bad;
    }
#pragma omp parallel for schedule(static) reduction(+ : bad_range, bad_mult, bad_err)
    for (int64_t i = 0; i < (1LL << 32); i++) {
        int32_t dg[3];
        or_decompose((uint32_t)i, 3, 7, dg);
        for (int j = 0; j < 3; j++)
            if (dg[j] < -64 || dg[j] >= 64) bad_range++;
        const int64_t rec = (int64_t)dg[0] * (1LL << 25) + (int64_t)dg[1] * (1LL << 18) + (int64_t)dg[2] * (1LL << 11);
        if (centred(rec, 1LL << 11) != 0) bad_mult++;
        const int64_t e = centred(i - rec, 1LL << 32);
        if (e < -(1LL << 10) || e >= (1LL << 10)) bad_err++;
    }
    printf("modswitch 2N=1024 %lld\nmodswitch 2N=2048 %lld\ndigit range %lld\nmultiple of 2^11 %lld\n"
           "nearest, ties up %lld\n",
           bad_ms[0], bad_ms[1], bad_range, bad_mult, bad_err);
    return (bad_ms[0] | bad_ms[1] | bad_range | bad_mult | bad_err) ? 1 : 0;
}
