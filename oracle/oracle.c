/*
 * CPU oracle for batched TFHE gate bootstrapping (test infrastructure).
 *
 * This file is TEST INFRASTRUCTURE. Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load or call it. The product path
 * (the HIP library) shares no code, header, table or constant generator with
 * it, and never calls it.
 *
 * What it computes (CryptoEmu, arXiv 2101.03403): every functional unit of the
 * emulator is a circuit of bootstrapped TFHE gates (Sec. 3, Table
 * "TFHEbenchmark"; homomorphic correctness f(a,b) = Dec(g(Enc a, Enc b)) in
 * Sec. 2). The paper treats the gate as a black box and cites the TFHE papers
 * (Chillotti, Gama, Georgieva, Izabachene) for it, so each step below is the
 * standard TFHE gate-bootstrapping definition written out plainly:
 *   gate linear combination -> modulus switch to Z/2N -> blind rotation of n
 *   CMux steps (external products TRGSW x TRLWE, signed gadget decomposition,
 *   negacyclic products mod X^N+1 over Torus32) -> sample extraction ->
 *   key switching.
 * Everything is exact uint32 arithmetic with wraparound (the torus T = R/Z is
 * represented by Z/2^32). Products are the schoolbook definition; there is no
 * FFT, no blocking and no fusion.
 *
 * Randomness: both sides implement the counter-based generator Philox4x32-10
 * (Salmon, Moraes, Dror, Shaw, SC'11) from its published definition, and use
 * the same counter assignment (stated at or_keygen and or_lwe_encrypt). The Gaussian
 * is the Box-Muller transform evaluated in IEEE double.
 *
 * Build: gcc -O3 -fopenmp -ffp-contract=off -fPIC -shared oracle.c -lm
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int32_t n;        /* LWE dimension of gate ciphertexts                */
    int32_t N;        /* TRLWE ring degree (power of two)                 */
    int32_t k;        /* TRLWE mask size; only k = 1 is supported         */
    int32_t l;        /* gadget decomposition length of the BK            */
    int32_t bgbit;    /* log2 of the gadget base Bg                       */
    int32_t t;        /* key-switching decomposition length              */
    int32_t basebit;  /* log2 of the key-switching base                   */
    int32_t pad;
    double sigma_lwe; /* std dev of fresh LWE noise, as a torus fraction  */
    double sigma_ks;  /* std dev of key-switching key noise              */
    double sigma_bk;  /* std dev of bootstrapping key noise              */
} or_params;

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., "Parallel random numbers: as easy as 1, 2, 3",
 * SC'11): 10 rounds of a multiply-xor Feistel-like bijection on a 128-bit
 * counter, keyed by a 64-bit key bumped by Weyl constants between rounds.   */
void or_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; round++) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Counter domains (fourth counter word). */
enum {
    OR_DOM_LWE_KEY = 1, OR_DOM_TLWE_KEY = 2, OR_DOM_BK_MASK = 3, OR_DOM_BK_NOISE = 4,
    OR_DOM_KS_MASK = 5, OR_DOM_KS_NOISE = 6, OR_DOM_ENC_MASK = 7, OR_DOM_ENC_NOISE = 8
};

static void or_block(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t dom, uint32_t out[4])
{
    uint32_t ctr[4] = { c0, c1, c2, dom };
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    or_philox4x32_10(ctr, key, out);
}

/* Box-Muller on one Philox block: two 53-bit uniforms u1 in (0,1], u2 in
 * [0,1); z = sqrt(-2 ln u1) cos(2 pi u2) is standard normal. Returned value is
 * the noise in units of 2^-32, rounded to the nearest integer. */
int64_t or_gauss_from_block(const uint32_t w[4], double sigma)
{
    uint64_t x1 = ((uint64_t)(w[0] >> 5) << 26) | (uint64_t)(w[1] >> 6);
    uint64_t x2 = ((uint64_t)(w[2] >> 5) << 26) | (uint64_t)(w[3] >> 6);
    double u1 = (double)(x1 + 1u) * 0x1.0p-53;
    double u2 = (double)x2 * 0x1.0p-53;
    double two_pi = 6.283185307179586;
    double z = sqrt(-2.0 * log(u1)) * cos(two_pi * u2);
    double scale = sigma * 4294967296.0;
    return llround(z * scale);
}

/* ------------------------------------------------------------------------ */
/* Negacyclic product in Z_{2^32}[X]/(X^N+1), schoolbook:
 *   (P*Q)_m = sum_{i+j=m} P_i Q_j - sum_{i+j=m+N} P_i Q_j   (mod 2^32).     */
void or_negacyclic_mul(int32_t N, const uint32_t *P, const uint32_t *Q, uint32_t *out)
{
    uint32_t *acc = (uint32_t *)calloc((size_t)N, sizeof(uint32_t));
    for (int32_t i = 0; i < N; i++) {
        uint32_t pi = P[i];
        for (int32_t j = 0; j < N - i; j++) acc[i + j] += pi * Q[j];
        for (int32_t j = N - i; j < N; j++) acc[i + j - N] -= pi * Q[j];
    }
    memcpy(out, acc, (size_t)N * sizeof(uint32_t));
    free(acc);
}

/* out += P*Q (negacyclic), same definition. */
static void or_negacyclic_muladd(int32_t N, const uint32_t *P, const uint32_t *Q, uint32_t *out)
{
    for (int32_t i = 0; i < N; i++) {
        uint32_t pi = P[i];
        for (int32_t j = 0; j < N - i; j++) out[i + j] += pi * Q[j];
        for (int32_t j = N - i; j < N; j++) out[i + j - N] -= pi * Q[j];
    }
}

/* Multiplication by the monomial X^a, a in [0, 2N): X^N = -1. */
void or_rotate(int32_t N, int32_t a, const uint32_t *P, uint32_t *out)
{
    for (int32_t m = 0; m < N; m++) {
        /* X^a * P_j X^j contributes to coefficient (j + a) mod 2N. */
        int32_t src = m - a;              /* j with j + a = m (mod 2N)     */
        int32_t sign = 1;
        while (src < 0) { src += N; sign = -sign; }
        out[m] = sign > 0 ? P[src] : (uint32_t)(0u - P[src]);
    }
}

/* Modulus switch of a torus element to Z/2N: the nearest integer to
 * x * 2N / 2^32, reduced mod 2N (ties round up). Computed in 64 bits. */
int32_t or_modswitch(uint32_t x, int32_t two_n)
{
    uint64_t num = (uint64_t)x * (uint64_t)two_n + (1ull << 31);
    return (int32_t)((num >> 32) % (uint64_t)two_n);
}

/* Signed gadget decomposition of a torus element with base Bg = 2^bgbit and l
 * levels: round x to the nearest multiple of 2^(32 - l*bgbit) (ties up), then
 * write the rounded value in balanced base Bg with digits in [-Bg/2, Bg/2),
 * so that sum_j d_j * 2^(32 - j*bgbit) = rounded x (mod 2^32), j = 1..l.
 * digits[j-1] receives d_j (d_1 is the most significant digit). */
void or_decompose(uint32_t x, int32_t l, int32_t bgbit, int32_t *digits)
{
    int32_t total = l * bgbit;
    uint64_t xr;
    if (total >= 32) {
        xr = x;
    } else {
        /* nearest integer to x / 2^(32-total), kept modulo 2^total */
        uint64_t shifted = ((uint64_t)x + (1ull << (31 - total))) >> (32 - total);
        xr = shifted & ((1ull << total) - 1);
    }
    int64_t bg = (int64_t)1 << bgbit;
    int64_t v = (int64_t)xr;
    for (int32_t j = l; j >= 1; j--) {      /* least significant digit first */
        int64_t r = v % bg;                 /* v >= 0 here                    */
        if (r >= bg / 2) r -= bg;
        digits[j - 1] = (int32_t)r;
        v = (v - r) / bg;                   /* exact, and v stays >= 0        */
    }
    /* any carry left in v is a multiple of 2^32 after scaling: dropped */
}

/* ------------------------------------------------------------------------ */
/* Key generation.
 *  lwe_key[n]   : LWE key s in {0,1}^n      bit = Philox(seed,(u,0,0,1)).w0 & 1
 *  tlwe_key[N]  : TRLWE key S in {0,1}[X]   bit = Philox(seed,(m,0,0,2)).w0 & 1
 *  bk[n][2l][2][N] : BK_i = TRGSW_S(s_i). Row r = c*l + j (c = 0: mask part,
 *      c = 1: body part), component q = 0 (A) / 1 (B).
 *      A_m = Philox(seed,(m,r,i,3)).w0, E_m = gauss(Philox(seed,(m,r,i,4)), sigma_bk),
 *      B = A*S + E, then s_i * 2^(32-(j+1)*bgbit) is added to the constant
 *      coefficient of component c.
 *  ksk[N][t][base][n+1] : KS[i][j][v] = LWE_s encryption of
 *      v * S_i * 2^(32-(j+1)*basebit); mask a_u = Philox(seed,(u, j*base+v, i, 5)).w0,
 *      noise = gauss(Philox(seed,(0, j*base+v, i, 6)), sigma_ks).              */
void or_keygen(const or_params *p, uint64_t seed, int32_t *lwe_key, int32_t *tlwe_key,
               uint32_t *bk, uint32_t *ksk)
{
    const int32_t n = p->n, N = p->N, l = p->l, t = p->t, base = 1 << p->basebit;
    uint32_t w[4];
    for (int32_t u = 0; u < n; u++) { or_block(seed, (uint32_t)u, 0, 0, OR_DOM_LWE_KEY, w); lwe_key[u] = (int32_t)(w[0] & 1u); }
    for (int32_t m = 0; m < N; m++) { or_block(seed, (uint32_t)m, 0, 0, OR_DOM_TLWE_KEY, w); tlwe_key[m] = (int32_t)(w[0] & 1u); }

    uint32_t *S = (uint32_t *)malloc((size_t)N * sizeof(uint32_t));
    for (int32_t m = 0; m < N; m++) S[m] = (uint32_t)tlwe_key[m];

    #pragma omp parallel for schedule(dynamic) collapse(2)
    for (int32_t i = 0; i < n; i++) {
        for (int32_t r = 0; r < 2 * l; r++) {
            uint32_t wb[4];
            uint32_t *A = bk + (((size_t)i * 2 * l + r) * 2 + 0) * N;
            uint32_t *B = bk + (((size_t)i * 2 * l + r) * 2 + 1) * N;
            for (int32_t m = 0; m < N; m++) {
                or_block(seed, (uint32_t)m, (uint32_t)r, (uint32_t)i, OR_DOM_BK_MASK, wb);
                A[m] = wb[0];
            }
            or_negacyclic_mul(N, A, S, B);
            for (int32_t m = 0; m < N; m++) {
                or_block(seed, (uint32_t)m, (uint32_t)r, (uint32_t)i, OR_DOM_BK_NOISE, wb);
                B[m] += (uint32_t)or_gauss_from_block(wb, p->sigma_bk);
            }
            int32_t c = r / l, j = r % l;
            uint32_t h = (uint32_t)1u << (32 - (j + 1) * p->bgbit);
            uint32_t mu = (uint32_t)lwe_key[i] * h;
            if (c == 0) A[0] += mu; else B[0] += mu;
        }
    }
    free(S);

    #pragma omp parallel for schedule(static) collapse(2)
    for (int32_t i = 0; i < N; i++) {
        for (int32_t j = 0; j < t; j++) {
            for (int32_t v = 0; v < base; v++) {
                uint32_t wk[4];
                uint32_t *row = ksk + (((size_t)i * t + j) * base + v) * (size_t)(n + 1);
                uint32_t body = 0;
                for (int32_t u = 0; u < n; u++) {
                    or_block(seed, (uint32_t)u, (uint32_t)(j * base + v), (uint32_t)i, OR_DOM_KS_MASK, wk);
                    row[u] = wk[0];
                    body += wk[0] * (uint32_t)lwe_key[u];
                }
                or_block(seed, 0, (uint32_t)(j * base + v), (uint32_t)i, OR_DOM_KS_NOISE, wk);
                uint32_t shift = (uint32_t)(32 - (j + 1) * p->basebit);
                uint32_t mu = (shift >= 32) ? 0u : (((uint32_t)v * (uint32_t)tlwe_key[i]) << shift);
                row[n] = body + mu + (uint32_t)or_gauss_from_block(wk, p->sigma_ks);
            }
        }
    }
}

/* LWE encryption of mu under key[dim] with encryption stream (seed, index):
 * a_u = Philox(seed,(u, idx_lo, idx_hi, 7)).w0, e = gauss(Philox(seed,(0, idx_lo, idx_hi, 8)), sigma),
 * b = <a, s> + mu + e. */
void or_lwe_encrypt(int32_t dim, const int32_t *key, uint64_t seed, uint64_t index,
                    uint32_t mu, double sigma, uint32_t *out)
{
    uint32_t w[4];
    uint32_t body = 0;
    for (int32_t u = 0; u < dim; u++) {
        or_block(seed, (uint32_t)u, (uint32_t)index, (uint32_t)(index >> 32), OR_DOM_ENC_MASK, w);
        out[u] = w[0];
        body += w[0] * (uint32_t)key[u];
    }
    or_block(seed, 0, (uint32_t)index, (uint32_t)(index >> 32), OR_DOM_ENC_NOISE, w);
    out[dim] = body + mu + (uint32_t)or_gauss_from_block(w, sigma);
}

/* Gate-bootstrapping encoding of a bit: true = +1/8, false = -1/8. */
void or_encrypt_bits(const or_params *p, const int32_t *lwe_key, uint64_t seed, uint64_t first_index,
                     const uint8_t *bits, int64_t count, uint32_t *out)
{
    #pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < count; e++) {
        uint32_t mu = bits[e] ? 0x20000000u : 0xE0000000u;
        or_lwe_encrypt(p->n, lwe_key, seed, first_index + (uint64_t)e, mu, p->sigma_lwe,
                       out + (size_t)e * (p->n + 1));
    }
}

/* Phase b - <a, s>. */
uint32_t or_lwe_phase(int32_t dim, const int32_t *key, const uint32_t *ct)
{
    uint32_t s = 0;
    for (int32_t u = 0; u < dim; u++) s += ct[u] * (uint32_t)key[u];
    return ct[dim] - s;
}

/* Decryption: the sign of the phase; phase 0 decrypts to false. */
void or_decrypt_bits(int32_t dim, const int32_t *key, const uint32_t *ct, int64_t count, uint8_t *bits)
{
    for (int64_t e = 0; e < count; e++)
        bits[e] = (int32_t)or_lwe_phase(dim, key, ct + (size_t)e * (dim + 1)) > 0 ? 1 : 0;
}

/* TRLWE phase B - A*S (k = 1). */
void or_tlwe_phase(int32_t N, const int32_t *tlwe_key, const uint32_t *acc, uint32_t *phase)
{
    uint32_t *S = (uint32_t *)malloc((size_t)N * sizeof(uint32_t));
    uint32_t *AS = (uint32_t *)malloc((size_t)N * sizeof(uint32_t));
    for (int32_t m = 0; m < N; m++) S[m] = (uint32_t)tlwe_key[m];
    or_negacyclic_mul(N, acc, S, AS);
    for (int32_t m = 0; m < N; m++) phase[m] = acc[N + m] - AS[m];
    free(S); free(AS);
}

/* ------------------------------------------------------------------------ */
/* Gate linear combination: c = (0,...,0,kappa) + w1*c1 + w2*c2 (mod 2^32).
 * op codes: 0 NAND, 1 AND, 2 OR, 3 XOR, 4 XNOR, 5 NOR, 6 ANDNY, 7 ANDYN,
 *           8 ORNY, 9 ORYN  (the bootstrapped binary gates of Table
 *           "TFHEbenchmark"). Returns -1 for an unknown op.                  */
int32_t or_gate_constants(int32_t op, uint32_t *kappa, int32_t *w1, int32_t *w2)
{
    const uint32_t P8 = 0x20000000u, M8 = 0xE0000000u, P4 = 0x40000000u, M4 = 0xC0000000u;
    switch (op) {
    case 0: *kappa = P8; *w1 = -1; *w2 = -1; return 0;   /* NAND  */
    case 1: *kappa = M8; *w1 = 1;  *w2 = 1;  return 0;   /* AND   */
    case 2: *kappa = P8; *w1 = 1;  *w2 = 1;  return 0;   /* OR    */
    case 3: *kappa = P4; *w1 = 2;  *w2 = 2;  return 0;   /* XOR   */
    case 4: *kappa = M4; *w1 = -2; *w2 = -2; return 0;   /* XNOR  */
    case 5: *kappa = M8; *w1 = -1; *w2 = -1; return 0;   /* NOR   */
    case 6: *kappa = M8; *w1 = -1; *w2 = 1;  return 0;   /* ANDNY: (not a) and b */
    case 7: *kappa = M8; *w1 = 1;  *w2 = -1; return 0;   /* ANDYN: a and (not b) */
    case 8: *kappa = P8; *w1 = -1; *w2 = 1;  return 0;   /* ORNY:  (not a) or b  */
    case 9: *kappa = P8; *w1 = 1;  *w2 = -1; return 0;   /* ORYN:  a or (not b)  */
    default: return -1;
    }
}

int32_t or_gate_lincomb(int32_t dim, int32_t op, const uint32_t *c1, const uint32_t *c2, uint32_t *out)
{
    uint32_t kappa; int32_t w1, w2;
    if (or_gate_constants(op, &kappa, &w1, &w2) != 0) return -1;
    for (int32_t u = 0; u <= dim; u++)
        out[u] = (uint32_t)w1 * c1[u] + (uint32_t)w2 * c2[u];
    out[dim] += kappa;
    return 0;
}

/* Blind rotation of a mod-switched LWE sample bar[0..n] (bar[n] = b-bar):
 *   ACC <- (0, X^{-bbar} v),   v = sum_j (1/8) X^j
 *   for i in 0..n-1:  ACC <- ACC + BK_i [external product] (X^{abar_i} ACC - ACC)
 * The external product decomposes each component of D = X^a ACC - ACC into l
 * signed digits and sums d_{c,j} * BK_i[c*l+j] over both output components.
 * acc_out: [2][N] (A then B). */
void or_blind_rotate(const or_params *p, const uint32_t *bk, const int32_t *bar, uint32_t *acc_out)
{
    const int32_t n = p->n, N = p->N, l = p->l;
    uint32_t *A = acc_out, *B = acc_out + N;
    uint32_t *v = (uint32_t *)malloc((size_t)N * sizeof(uint32_t));
    uint32_t *rot = (uint32_t *)malloc((size_t)N * sizeof(uint32_t));
    uint32_t *D = (uint32_t *)malloc((size_t)2 * N * sizeof(uint32_t));
    uint32_t *dig = (uint32_t *)malloc((size_t)2 * l * N * sizeof(uint32_t));
    int32_t *dj = (int32_t *)malloc((size_t)l * sizeof(int32_t));

    for (int32_t m = 0; m < N; m++) v[m] = 0x20000000u;
    memset(A, 0, (size_t)N * sizeof(uint32_t));
    or_rotate(N, (2 * N - bar[n]) % (2 * N), v, B);

    for (int32_t i = 0; i < n; i++) {
        /* D = X^{abar_i} * ACC - ACC, component-wise */
        for (int32_t c = 0; c < 2; c++) {
            const uint32_t *src = c == 0 ? A : B;
            or_rotate(N, bar[i], src, rot);
            for (int32_t m = 0; m < N; m++) D[c * N + m] = rot[m] - src[m];
        }
        /* gadget decomposition: dig[(c*l + j)][m] */
        for (int32_t c = 0; c < 2; c++)
            for (int32_t m = 0; m < N; m++) {
                or_decompose(D[c * N + m], l, p->bgbit, dj);
                for (int32_t j = 0; j < l; j++) dig[((size_t)c * l + j) * N + m] = (uint32_t)dj[j];
            }
        /* ACC += sum_{row} dig_row * BK_i[row]  (both components) */
        for (int32_t r = 0; r < 2 * l; r++) {
            const uint32_t *bkA = bk + (((size_t)i * 2 * l + r) * 2 + 0) * N;
            const uint32_t *bkB = bk + (((size_t)i * 2 * l + r) * 2 + 1) * N;
            or_negacyclic_muladd(N, dig + (size_t)r * N, bkA, A);
            or_negacyclic_muladd(N, dig + (size_t)r * N, bkB, B);
        }
    }
    free(v); free(rot); free(D); free(dig); free(dj);
}

/* Sample extraction of the constant coefficient: an LWE sample of dimension N
 * under the key made of the coefficients of S:
 *   a'_0 = A_0,  a'_j = -A_{N-j} (j >= 1),  b' = B_0. */
void or_sample_extract(int32_t N, const uint32_t *acc, uint32_t *out)
{
    out[0] = acc[0];
    for (int32_t j = 1; j < N; j++) out[j] = 0u - acc[N - j];
    out[N] = acc[N];
}

/* Key switching from dimension N to n: each a'_i is rounded to t*basebit bits
 * and written in unsigned base 2^basebit (most significant digit first); the
 * output is (0,...,0,b') - sum over nonzero digits of KS[i][j][digit]. */
void or_key_switch(const or_params *p, const uint32_t *ksk, const uint32_t *in, uint32_t *out)
{
    const int32_t n = p->n, N = p->N, t = p->t, bb = p->basebit, base = 1 << bb;
    const int32_t prec = t * bb;
    for (int32_t u = 0; u < n; u++) out[u] = 0;
    out[n] = in[N];
    for (int32_t i = 0; i < N; i++) {
        uint64_t xr;
        if (prec >= 32) xr = in[i];
        else xr = (((uint64_t)in[i] + (1ull << (31 - prec))) >> (32 - prec)) & ((1ull << prec) - 1);
        for (int32_t j = 0; j < t; j++) {
            int32_t d = (int32_t)((xr >> (prec - (j + 1) * bb)) & (uint64_t)(base - 1));
            if (d == 0) continue;
            const uint32_t *row = ksk + (((size_t)i * t + j) * base + d) * (size_t)(n + 1);
            for (int32_t u = 0; u <= n; u++) out[u] -= row[u];
        }
    }
}

/* One bootstrapped gate: lincomb, modulus switch, blind rotation, extraction,
 * key switch. extracted (nullable) receives the dimension-N sample. */
int32_t or_bootstrap_gate(const or_params *p, const uint32_t *bk, const uint32_t *ksk, int32_t op,
                          const uint32_t *c1, const uint32_t *c2, uint32_t *extracted, uint32_t *out)
{
    const int32_t n = p->n, N = p->N;
    uint32_t *lin = (uint32_t *)malloc((size_t)(n + 1) * sizeof(uint32_t));
    int32_t *bar = (int32_t *)malloc((size_t)(n + 1) * sizeof(int32_t));
    uint32_t *acc = (uint32_t *)malloc((size_t)2 * N * sizeof(uint32_t));
    uint32_t *ext = (uint32_t *)malloc((size_t)(N + 1) * sizeof(uint32_t));
    int32_t rc = or_gate_lincomb(n, op, c1, c2, lin);
    if (rc == 0) {
        for (int32_t u = 0; u <= n; u++) bar[u] = or_modswitch(lin[u], 2 * N);
        or_blind_rotate(p, bk, bar, acc);
        or_sample_extract(N, acc, ext);
        if (extracted) memcpy(extracted, ext, (size_t)(N + 1) * sizeof(uint32_t));
        if (out) or_key_switch(p, ksk, ext, out);
    }
    free(lin); free(bar); free(acc); free(ext);
    return rc;
}

/* Batch of independent gates, parallel across gates only.
 * c1s, c2s, outs: [B][n+1]; extracted (nullable): [B][N+1]; outs nullable. */
int32_t or_bootstrap_batch(const or_params *p, const uint32_t *bk, const uint32_t *ksk,
                           const int32_t *ops, const uint32_t *c1s, const uint32_t *c2s, int64_t count,
                           uint32_t *extracted, uint32_t *outs)
{
    const size_t n1 = (size_t)p->n + 1, N1 = (size_t)p->N + 1;
    int32_t bad = 0;
    #pragma omp parallel for schedule(dynamic, 1) reduction(|:bad)
    for (int64_t g = 0; g < count; g++) {
        int32_t rc = or_bootstrap_gate(p, bk, ksk, ops[g], c1s + g * n1, c2s + g * n1,
                                       extracted ? extracted + g * N1 : NULL, outs ? outs + g * n1 : NULL);
        if (rc) bad = 1;
    }
    return bad ? -1 : 0;
}

/* Blind rotation only, for a batch of already mod-switched samples. */
void or_blind_rotate_batch(const or_params *p, const uint32_t *bk, const int32_t *bars, int64_t count,
                           uint32_t *accs)
{
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t g = 0; g < count; g++)
        or_blind_rotate(p, bk, bars + g * (size_t)(p->n + 1), accs + g * (size_t)2 * p->N);
}

/* Key switch of a batch of dimension-N samples. */
void or_key_switch_batch(const or_params *p, const uint32_t *ksk, const uint32_t *ins, int64_t count, uint32_t *outs)
{
    #pragma omp parallel for schedule(static)
    for (int64_t g = 0; g < count; g++)
        or_key_switch(p, ksk, ins + g * (size_t)(p->N + 1), outs + g * (size_t)(p->n + 1));
}

/* Vector helpers used by the pins (plain loops over the scalar definitions). */
void or_modswitch_array(const uint32_t *x, int64_t count, int32_t two_n, int32_t *out)
{
    #pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < count; e++) out[e] = or_modswitch(x[e], two_n);
}

void or_decompose_array(const uint32_t *x, int64_t count, int32_t l, int32_t bgbit, int32_t *digits)
{
    #pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < count; e++) or_decompose(x[e], l, bgbit, digits + e * l);
}

void or_gauss_array(uint64_t seed, int64_t count, double sigma, int64_t *out)
{
    #pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < count; e++) {
        uint32_t w[4];
        or_block(seed, (uint32_t)e, (uint32_t)(e >> 32), 0, OR_DOM_ENC_NOISE, w);
        out[e] = or_gauss_from_block(w, sigma);
    }
}

/* Threads OpenMP will use for the batch routines. */
int32_t or_num_threads(void)
{
#ifdef _OPENMP
    return (int32_t)omp_get_max_threads();
#else
    return 1;
#endif
}
