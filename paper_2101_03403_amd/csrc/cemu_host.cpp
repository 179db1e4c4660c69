// Host part of libcemu: parameter sets, deterministic key generation,
// encryption, decryption, key export and error reporting.
//
// Key generation follows the TFHE gate-bootstrapping keyset that the paper's
// TFHE API generates before any gate evaluation (Sec. 3, "TFHE API"):
//   s in {0,1}^n (LWE key), S in {0,1}[X]/(X^N+1) (TRLWE key),
//   BK_i = TRGSW_S(s_i) for i < n, KS[i][j][v] = LWE_s(v * S_i / base^(j+1)).
// Randomness is the counter-based generator Philox4x32-10 (Salmon et al.,
// SC'11): every random word is the output at a counter fixed by what it is
// for, keyed by the user seed, so generation order and threading do not
// change the keys:
//   LWE key bit u        : ctr (u, 0, 0, 1), word 0, bit 0
//   TRLWE key bit m      : ctr (m, 0, 0, 2), word 0, bit 0
//   BK mask  (i, r, m)   : ctr (m, r, i, 3), word 0
//   BK noise (i, r, m)   : ctr (m, r, i, 4), Box-Muller on the four words
//   KS mask  (i, j, v, u): ctr (u, j*base+v, i, 5), word 0
//   KS noise (i, j, v)   : ctr (0, j*base+v, i, 6)
//   encryption e, mask u : ctr (u, e_lo, e_hi, 7) keyed by the encryption seed
//   encryption e, noise  : ctr (0, e_lo, e_hi, 8)
// The Gaussian is Box-Muller in IEEE double: u1 = (x1+1)/2^53 in (0,1],
// u2 = x2/2^53 with x1 = (w0>>5)*2^26 + (w1>>6), x2 likewise from (w2, w3);
// z = sqrt(-2 ln u1) cos(2 pi u2); noise = nearest integer to z*sigma*2^32.
// This file is compiled without floating-point contraction so the double
// arithmetic is the plain sequence of IEEE operations.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <exception>
#include <memory>
#include <mutex>
#include <new>
#include <thread>

#include "cemu_internal.h"

namespace cemu {

namespace {
thread_local std::string g_last_error;
}

int fail(int code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

void clear_error() { g_last_error.clear(); }

int check_params(const cemu_params *p)
{
    if (!p) return fail(CEMU_ERR_NULL, "params is NULL");
    if (p->k != 1) return fail(CEMU_ERR_UNSUPPORTED, "only k = 1 is supported");
    if (p->N != 512 && p->N != 1024) return fail(CEMU_ERR_UNSUPPORTED, "N must be 512 or 1024");
    if (p->n < 1 || p->n > CEMU_MAX_LWE_N) return fail(CEMU_ERR_PARAM, "n must be in [1, 4096]");
    if (p->n > CEMU_MAX_KEY_N)
        return fail(CEMU_ERR_UNSUPPORTED, "keys need n <= 767 (the key switch writes n + 1 <= 768 columns)");
    if (p->l != 3 || p->bgbit != 7)
        return fail(CEMU_ERR_UNSUPPORTED, "the kernels need l = 3 and Bgbit = 7 (signed 7-bit digits)");
    if (p->basebit != 2) return fail(CEMU_ERR_UNSUPPORTED, "key switching needs basebit = 2");
    if (p->t < 1 || p->t * p->basebit > 32) return fail(CEMU_ERR_PARAM, "t must satisfy 1 <= t, t*basebit <= 32");
    // a deviation of a whole torus period or more (or NaN, or infinity) has
    // no meaning, and its samples would overflow the rounding to an integer
    auto ok_sigma = [](double s) { return s >= 0.0 && s <= 1.0; };
    if (!ok_sigma(p->sigma_lwe) || !ok_sigma(p->sigma_ks) || !ok_sigma(p->sigma_bk))
        return fail(CEMU_ERR_PARAM, "noise deviations must be in [0, 1] (torus units)");
    return CEMU_OK;
}

namespace {

// ---------------------------------------------------------------- Philox4x32-10
struct Philox {
    uint32_t k0, k1;
    explicit Philox(uint64_t seed) : k0((uint32_t)seed), k1((uint32_t)(seed >> 32)) {}

    // One 128-bit output block for the 128-bit counter (x0, x1, x2, x3).
    void block(uint32_t x0, uint32_t x1, uint32_t x2, uint32_t x3, uint32_t out[4]) const
    {
        static constexpr uint32_t kMulA = 0xD2511F53u, kMulB = 0xCD9E8D57u;
        static constexpr uint32_t kWeylA = 0x9E3779B9u, kWeylB = 0xBB67AE85u;
        uint32_t key0 = k0, key1 = k1;
        uint32_t v[4] = {x0, x1, x2, x3};
        for (int r = 0; r < 10; ++r) {
            const uint64_t pa = (uint64_t)kMulA * v[0];
            const uint64_t pb = (uint64_t)kMulB * v[2];
            const uint32_t t0 = (uint32_t)(pb >> 32) ^ v[1] ^ key0;
            const uint32_t t2 = (uint32_t)(pa >> 32) ^ v[3] ^ key1;
            v[1] = (uint32_t)pb;
            v[3] = (uint32_t)pa;
            v[0] = t0;
            v[2] = t2;
            key0 += kWeylA;
            key1 += kWeylB;
        }
        std::memcpy(out, v, sizeof v);
    }
    uint32_t word(uint32_t x0, uint32_t x1, uint32_t x2, uint32_t x3) const
    {
        uint32_t o[4];
        block(x0, x1, x2, x3, o);
        return o[0];
    }
    // Torus noise of standard deviation sigma (torus units), as a uint32.
    uint32_t gauss(uint32_t x0, uint32_t x1, uint32_t x2, uint32_t x3, double sigma) const
    {
        if (sigma == 0.0) return 0u;
        uint32_t w[4];
        block(x0, x1, x2, x3, w);
        const uint64_t h1 = ((uint64_t)(w[0] >> 5) << 26) | (uint64_t)(w[1] >> 6);
        const uint64_t h2 = ((uint64_t)(w[2] >> 5) << 26) | (uint64_t)(w[3] >> 6);
        const double u1 = std::ldexp((double)(h1 + 1), -53);
        const double u2 = std::ldexp((double)h2, -53);
        const double radius = std::sqrt(-2.0 * std::log(u1));
        const double angle = 6.283185307179586 * u2;
        const double z = radius * std::cos(angle);
        const double scaled = z * (sigma * 4294967296.0);
        return (uint32_t)(int64_t)std::llround(scaled);
    }
};

enum : uint32_t {
    kDomLweKey = 1, kDomTlweKey = 2, kDomBkMask = 3, kDomBkNoise = 4,
    kDomKsMask = 5, kDomKsNoise = 6, kDomEncMask = 7, kDomEncNoise = 8
};

// Runs f(0 .. count-1) over the host's threads. An exception thrown by f is
// rethrown in the caller once every worker has stopped; slices for which no
// thread could be started run on the calling thread.
template <class F>
void parallel_for(int64_t count, F &&f)
{
    unsigned hw = std::thread::hardware_concurrency();
    int64_t nt = std::max<int64_t>(1, std::min<int64_t>(hw ? hw : 4, 32));
    nt = std::min(nt, count);
    if (nt <= 1) {
        for (int64_t i = 0; i < count; ++i) f(i);
        return;
    }
    std::exception_ptr err;
    std::mutex err_mu;
    auto slice = [&](int64_t w) {
        try {
            for (int64_t i = w; i < count; i += nt) f(i);
        } catch (...) {
            std::lock_guard<std::mutex> g(err_mu);
            if (!err) err = std::current_exception();
        }
    };
    std::vector<std::thread> th;
    int64_t w = 0;
    try {
        th.reserve((size_t)nt);
        for (; w < nt; ++w) th.emplace_back(slice, w);
    } catch (...) {
        for (; w < nt; ++w) slice(w);
    }
    for (auto &x : th) x.join();
    if (err) std::rethrow_exception(err);
}

// Runs the body of an entry point, turning a host exception (allocation
// failure above all) into an error code, so that none crosses the C ABI.
template <class F>
int guarded(F &&body)
{
    try {
        return body();
    } catch (const std::bad_alloc &) {
        return fail(CEMU_ERR_OOM, "host allocation failed");
    } catch (const std::exception &e) {
        return fail(CEMU_ERR_OOM, std::string("host error: ") + e.what());
    } catch (...) {
        return fail(CEMU_ERR_OOM, "host error");
    }
}

// Signed balanced 8-bit limbs of a Torus32 value: x = sum_k 2^(8k) s_k mod 2^32,
// s_k in [-128, 127].
inline void limbs4(uint32_t x, int8_t s[4])
{
    uint32_t y = x;
    for (int k = 0; k < 4; ++k) {
        const int8_t lo = (int8_t)(uint8_t)(y & 0xFFu);
        s[k] = lo;
        y = (y - (uint32_t)(int32_t)lo) >> 8;
    }
}

inline uint32_t unlimbs4(const int8_t s[4])
{
    uint32_t x = 0;
    for (int k = 3; k >= 0; --k) x = (x << 8) + (uint32_t)(int32_t)s[k];
    return x;
}

// LWE encryption of mu under key (dimension d) with the encryption stream.
void lwe_encrypt(const int32_t *key, int32_t d, const Philox &rng, uint64_t index, uint32_t mu, double sigma,
                 uint32_t *out)
{
    const uint32_t ilo = (uint32_t)index, ihi = (uint32_t)(index >> 32);
    uint32_t body = mu;
    for (int32_t u = 0; u < d; ++u) {
        const uint32_t a = rng.word((uint32_t)u, ilo, ihi, kDomEncMask);
        out[u] = a;
        if (key[u]) body += a;
    }
    out[d] = body + rng.gauss(0, ilo, ihi, kDomEncNoise, sigma);
}

uint32_t phase_of(const int32_t *key, int32_t d, const uint32_t *ct)
{
    uint32_t s = 0;
    for (int32_t u = 0; u < d; ++u)
        if (key[u]) s += ct[u];
    return ct[d] - s;
}

}  // namespace
}  // namespace cemu

using namespace cemu;

extern "C" {

int cemu_params_default(cemu_params *p, int which)
{
    clear_error();
    if (!p) return fail(CEMU_ERR_NULL, "params is NULL");
    if (which != CEMU_STD && which != CEMU_TOY) return fail(CEMU_ERR_PARAM, "unknown parameter set");
    std::memset(p, 0, sizeof *p);
    p->n = which == CEMU_STD ? 630 : 256;
    p->N = which == CEMU_STD ? 1024 : 512;
    p->k = 1;
    p->l = 3;
    p->bgbit = 7;
    p->t = 8;
    p->basebit = 2;
    p->sigma_lwe = std::ldexp(1.0, -15);
    p->sigma_ks = std::ldexp(1.0, -15);
    p->sigma_bk = std::ldexp(1.0, -25);
    return CEMU_OK;
}

int cemu_keygen(const cemu_params *p, uint64_t seed, cemu_secret_key **sk_out, cemu_cloud_key **ck_out)
{
    clear_error();
    if (!sk_out || !ck_out) return fail(CEMU_ERR_NULL, "output handle pointer is NULL");
    *sk_out = nullptr;
    *ck_out = nullptr;
    const int rc = check_params(p);
    if (rc) return rc;
    return guarded([&]() -> int {
        const int32_t n = p->n, N = p->N, l = p->l, t = p->t, base = 1 << p->basebit;
        const Philox rng(seed);

        std::unique_ptr<cemu_secret_key> sk(new cemu_secret_key);
        sk->p = *p;
        sk->lwe_key.resize((size_t)n);
        sk->tlwe_key.resize((size_t)N);
        for (int32_t u = 0; u < n; ++u) sk->lwe_key[(size_t)u] = (int32_t)(rng.word((uint32_t)u, 0, 0, kDomLweKey) & 1u);
        for (int32_t m = 0; m < N; ++m) sk->tlwe_key[(size_t)m] = (int32_t)(rng.word((uint32_t)m, 0, 0, kDomTlweKey) & 1u);

        // Positions of the ones of S: A*S is the sum of X^k * A over them.
        std::vector<int32_t> ones;
        for (int32_t m = 0; m < N; ++m)
            if (sk->tlwe_key[(size_t)m]) ones.push_back(m);

        const size_t rbytes = (size_t)2 * N;
        std::vector<uint8_t> bk8((size_t)n * 2 * l * 2 * 4 * rbytes);
        std::vector<uint32_t> ksk((size_t)N * t * base * (n + 1));
        // TRGSW rows: one task per (i, r).
        parallel_for((int64_t)n * 2 * l, [&](int64_t task) {
            const int32_t i = (int32_t)(task / (2 * l)), r = (int32_t)(task % (2 * l));
            std::vector<uint32_t> A((size_t)N), B((size_t)N, 0u);
            for (int32_t m = 0; m < N; ++m) A[(size_t)m] = rng.word((uint32_t)m, (uint32_t)r, (uint32_t)i, kDomBkMask);
            for (int32_t k : ones) {          // B += X^k * A
                for (int32_t m = 0; m < N; ++m) {
                    const int32_t src = m - k;
                    B[(size_t)m] += src >= 0 ? A[(size_t)src] : 0u - A[(size_t)(src + N)];
                }
            }
            for (int32_t m = 0; m < N; ++m)
                B[(size_t)m] += rng.gauss((uint32_t)m, (uint32_t)r, (uint32_t)i, kDomBkNoise, p->sigma_bk);
            const int32_t c = r / l, j = r % l;
            if (sk->lwe_key[(size_t)i]) {
                const uint32_t h = 1u << (32 - (j + 1) * p->bgbit);
                if (c == 0) A[0] += h; else B[0] += h;
            }
            // int8-limb layout of both components
            for (int q = 0; q < 2; ++q) {
                const std::vector<uint32_t> &P = q == 0 ? A : B;
                uint8_t *dst = bk8.data() + (((size_t)i * 2 * l + r) * 2 + q) * 4 * rbytes;
                for (int32_t u = 0; u < 2 * N; ++u) {
                    const int32_t e = 2 * N - 1 - u;  // index into the extended sequence
                    const uint32_t val = e >= N ? P[(size_t)(e - N)] : 0u - P[(size_t)e];
                    int8_t s[4];
                    limbs4(val, s);
                    for (int kk = 0; kk < 4; ++kk) dst[(size_t)kk * rbytes + (size_t)u] = (uint8_t)s[kk];
                }
            }
        });

        // Key-switching key: one task per (i, j).
        parallel_for((int64_t)N * t, [&](int64_t task) {
            const int32_t i = (int32_t)(task / t), j = (int32_t)(task % t);
            for (int32_t v = 0; v < base; ++v) {
                uint32_t *row = ksk.data() + (((size_t)i * t + j) * base + v) * (size_t)(n + 1);
                const uint32_t c1 = (uint32_t)(j * base + v);
                uint32_t body = 0;
                for (int32_t u = 0; u < n; ++u) {
                    const uint32_t a = rng.word((uint32_t)u, c1, (uint32_t)i, kDomKsMask);
                    row[u] = a;
                    if (sk->lwe_key[(size_t)u]) body += a;
                }
                const int32_t sh = 32 - (j + 1) * p->basebit;
                const uint32_t mu = sh >= 32 ? 0u : ((uint32_t)(v * sk->tlwe_key[(size_t)i]) << sh);
                row[n] = body + mu + rng.gauss(0, c1, (uint32_t)i, kDomKsNoise, p->sigma_ks);
            }
        });

        std::vector<uint8_t> ksk_mfma;
        if (ks_mfma_supported(*p)) {
            ksk_mfma.resize(ks_mfma_bytes(*p));
            const int ntiles = ks_mfma_ntiles(*p);
            parallel_for((int64_t)4 * ntiles, [&](int64_t task) {
                ks_mfma_arrange(*p, ksk.data(), ksk_mfma.data(), (int)(task / ntiles), (int)(task % ntiles));
            });
        }

        // device buffers are released with the handle on every failure path
        struct CloudDel {
            void operator()(cemu_cloud_key *c) const
            {
                release_cloud_key(c);
                delete c;
            }
        };
        std::unique_ptr<cemu_cloud_key, CloudDel> ck(new cemu_cloud_key);
        ck->p = *p;
        const int up = upload_cloud_key(ck.get(), bk8, ksk, ksk_mfma);
        if (up) return up;
        *sk_out = sk.release();
        *ck_out = ck.release();
        return CEMU_OK;
    });
}

int cemu_secret_params(const cemu_secret_key *sk, cemu_params *p)
{
    clear_error();
    if (!sk || !p) return fail(CEMU_ERR_NULL, "NULL argument");
    *p = sk->p;
    return CEMU_OK;
}

int cemu_cloud_params(const cemu_cloud_key *ck, cemu_params *p)
{
    clear_error();
    if (!ck || !p) return fail(CEMU_ERR_NULL, "NULL argument");
    *p = ck->p;
    return CEMU_OK;
}

int cemu_encrypt(const cemu_secret_key *sk, const uint8_t *bits, int64_t count, uint64_t seed,
                 uint64_t first_index, uint32_t *out)
{
    clear_error();
    if (!sk || (count > 0 && (!bits || !out))) return fail(CEMU_ERR_NULL, "NULL argument");
    if (count < 0) return fail(CEMU_ERR_RANGE, "count < 0");
    const Philox rng(seed);
    const int32_t n = sk->p.n;
    return guarded([&]() -> int {
        parallel_for(count, [&](int64_t e) {
            const uint32_t mu = bits[e] ? 0x20000000u : 0xE0000000u;
            lwe_encrypt(sk->lwe_key.data(), n, rng, first_index + (uint64_t)e, mu, sk->p.sigma_lwe,
                        out + (size_t)e * (size_t)(n + 1));
        });
        return CEMU_OK;
    });
}

int cemu_phase(const cemu_secret_key *sk, int extracted, const uint32_t *ct, int64_t count, uint32_t *phase)
{
    clear_error();
    if (!sk || (count > 0 && (!ct || !phase))) return fail(CEMU_ERR_NULL, "NULL argument");
    if (count < 0) return fail(CEMU_ERR_RANGE, "count < 0");
    const int32_t d = extracted ? sk->p.N : sk->p.n;
    const int32_t *key = extracted ? sk->tlwe_key.data() : sk->lwe_key.data();
    for (int64_t e = 0; e < count; ++e) phase[e] = phase_of(key, d, ct + (size_t)e * (size_t)(d + 1));
    return CEMU_OK;
}

int cemu_decrypt(const cemu_secret_key *sk, const uint32_t *ct, int64_t count, uint8_t *bits)
{
    clear_error();
    if (!sk || (count > 0 && (!ct || !bits))) return fail(CEMU_ERR_NULL, "NULL argument");
    if (count < 0) return fail(CEMU_ERR_RANGE, "count < 0");
    const int32_t n = sk->p.n;
    for (int64_t e = 0; e < count; ++e)
        bits[e] = (int32_t)phase_of(sk->lwe_key.data(), n, ct + (size_t)e * (size_t)(n + 1)) > 0 ? 1 : 0;
    return CEMU_OK;
}

int cemu_decrypt_extracted(const cemu_secret_key *sk, const uint32_t *ct, int64_t count, uint8_t *bits)
{
    clear_error();
    if (!sk || (count > 0 && (!ct || !bits))) return fail(CEMU_ERR_NULL, "NULL argument");
    if (count < 0) return fail(CEMU_ERR_RANGE, "count < 0");
    const int32_t N = sk->p.N;
    for (int64_t e = 0; e < count; ++e)
        bits[e] = (int32_t)phase_of(sk->tlwe_key.data(), N, ct + (size_t)e * (size_t)(N + 1)) > 0 ? 1 : 0;
    return CEMU_OK;
}

int cemu_export_keys(const cemu_secret_key *sk, const cemu_cloud_key *ck, int32_t *lwe_key, int32_t *tlwe_key,
                     uint32_t *bk, uint32_t *ksk)
{
    clear_error();
    if ((lwe_key || tlwe_key) && !sk) return fail(CEMU_ERR_NULL, "secret key is NULL");
    if ((bk || ksk) && !ck) return fail(CEMU_ERR_NULL, "cloud key is NULL");
    return guarded([&]() -> int {
        if (lwe_key) std::memcpy(lwe_key, sk->lwe_key.data(), sk->lwe_key.size() * sizeof(int32_t));
        if (tlwe_key) std::memcpy(tlwe_key, sk->tlwe_key.data(), sk->tlwe_key.size() * sizeof(int32_t));
        if (bk) {
            std::vector<uint8_t> bk8;
            int rc = download_bk8(ck, bk8);
            if (rc) return rc;
            const int32_t n = ck->p.n, N = ck->p.N, l = ck->p.l;
            const size_t rbytes = (size_t)2 * N;
            for (int32_t i = 0; i < n; ++i)
                for (int32_t r = 0; r < 2 * l; ++r)
                    for (int q = 0; q < 2; ++q) {
                        const uint8_t *src = bk8.data() + (((size_t)i * 2 * l + r) * 2 + q) * 4 * rbytes;
                        uint32_t *dst = bk + (((size_t)i * 2 * l + r) * 2 + q) * (size_t)N;
                        for (int32_t m = 0; m < N; ++m) {
                            // BK[m] sits at extended index N + m, i.e. u = N - 1 - m
                            const size_t u = (size_t)(N - 1 - m);
                            int8_t s[4];
                            for (int kk = 0; kk < 4; ++kk) s[kk] = (int8_t)src[(size_t)kk * rbytes + u];
                            dst[m] = unlimbs4(s);
                        }
                    }
        }
        if (ksk) {
            std::vector<uint32_t> k;
            int rc = download_ksk(ck, k);
            if (rc) return rc;
            std::memcpy(ksk, k.data(), k.size() * sizeof(uint32_t));
        }
        return CEMU_OK;
    });
}

void cemu_free_secret_key(cemu_secret_key *sk) { delete sk; }

void cemu_free_cloud_key(cemu_cloud_key *ck)
{
    if (!ck) return;
    release_cloud_key(ck);
    delete ck;
}

const char *cemu_last_error(void) { return g_last_error.c_str(); }

const char *cemu_version(void) { return "cemu 0.1 (gfx950)"; }

}  // extern "C"
