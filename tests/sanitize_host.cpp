// Driver for running the library's host code (cemu_host.cpp: parameters,
// key generation, encryption, decryption, phases, key export, argument
// checks) under AddressSanitizer and UndefinedBehaviorSanitizer without a
// GPU (test infrastructure; built by tests/test_sanitizers.py with g++).
//
// The device side of key generation is replaced by the stand-ins below: the
// "upload" keeps host copies of the key layouts and the "download" returns
// them, so cemu_export_keys reads back, and recombines, exactly the int8
// limbs key generation produced. The key-switching key's MFMA layout (built
// by device-side code) is reported unsupported here. The exported keys and
// the encryptions are compared with the CPU oracle's, which is linked in as
// an independent implementation. Returns the number of failed checks.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../paper_2101_03403_amd/csrc/cemu_internal.h"

extern "C" {
struct or_params {
    int32_t n, N, k, l, bgbit, t, basebit, pad;
    double sigma_lwe, sigma_ks, sigma_bk;
};
void or_keygen(const or_params *p, uint64_t seed, int32_t *lwe_key, int32_t *tlwe_key, uint32_t *bk, uint32_t *ksk);
void or_encrypt_bits(const or_params *p, const int32_t *lwe_key, uint64_t seed, uint64_t first_index,
                     const uint8_t *bits, int64_t count, uint32_t *out);
uint32_t or_lwe_phase(int32_t dim, const int32_t *key, const uint32_t *ct);
}

namespace {
struct HostCopies {
    std::vector<uint8_t> bk8;
    std::vector<uint32_t> ksk;
};
std::vector<std::pair<const cemu_cloud_key *, HostCopies>> g_keys;

HostCopies *find(const cemu_cloud_key *ck)
{
    for (auto &e : g_keys)
        if (e.first == ck) return &e.second;
    return nullptr;
}
}  // namespace

namespace cemu {
int upload_cloud_key(cemu_cloud_key *ck, const std::vector<uint8_t> &bk8, const std::vector<uint32_t> &ksk,
                     const std::vector<uint8_t> &)
{
    ck->device = 0;
    g_keys.push_back({ck, HostCopies{bk8, ksk}});
    return CEMU_OK;
}
int download_bk8(const cemu_cloud_key *ck, std::vector<uint8_t> &bk8)
{
    HostCopies *h = find(ck);
    if (!h) return fail(CEMU_ERR_PARAM, "unknown key");
    bk8 = h->bk8;
    return CEMU_OK;
}
int download_ksk(const cemu_cloud_key *ck, std::vector<uint32_t> &ksk)
{
    HostCopies *h = find(ck);
    if (!h) return fail(CEMU_ERR_PARAM, "unknown key");
    ksk = h->ksk;
    return CEMU_OK;
}
void release_cloud_key(cemu_cloud_key *ck)
{
    for (size_t i = 0; i < g_keys.size(); ++i)
        if (g_keys[i].first == ck) {
            g_keys.erase(g_keys.begin() + (long)i);
            return;
        }
}
bool ks_mfma_supported(const cemu_params &) { return false; }
size_t ks_mfma_bytes(const cemu_params &) { return 0; }
int ks_mfma_ntiles(const cemu_params &) { return 0; }
void ks_mfma_arrange(const cemu_params &, const uint32_t *, uint8_t *, int, int) {}
}  // namespace cemu

static int failures = 0;

static void check(bool ok, const char *what)
{
    if (!ok) {
        std::fprintf(stderr, "FAILED: %s\n", what);
        failures++;
    }
}

int main()
{
    cemu_params p;
    check(cemu_params_default(&p, CEMU_TOY) == CEMU_OK, "toy parameters");
    check(cemu_params_default(nullptr, CEMU_TOY) == CEMU_ERR_NULL, "null parameters");
    check(cemu_params_default(&p, 9) == CEMU_ERR_PARAM, "unknown parameter set");
    check(cemu_params_default(&p, CEMU_TOY) == CEMU_OK, "toy parameters again");
    const int32_t n = p.n, N = p.N, n1 = n + 1, N1 = N + 1;

    cemu_secret_key *sk = nullptr;
    cemu_cloud_key *ck = nullptr;
    cemu_params bad = p;
    bad.n = 768;
    check(cemu_keygen(&bad, 1, &sk, &ck) == CEMU_ERR_UNSUPPORTED && !sk && !ck, "n beyond the key switch refused");
    check(cemu_keygen(&p, 2021, &sk, &ck) == CEMU_OK && sk && ck, "keygen");

    // keys against the oracle's
    const or_params op = {p.n, p.N, p.k, p.l, p.bgbit, p.t, p.basebit, 0, p.sigma_lwe, p.sigma_ks, p.sigma_bk};
    const size_t bk_words = (size_t)n * 2 * p.l * 2 * N, ksk_words = (size_t)N * p.t * 4 * n1;
    std::vector<int32_t> lwe(n), tlwe(N), olwe(n), otlwe(N);
    std::vector<uint32_t> bk(bk_words), ksk(ksk_words), obk(bk_words), oksk(ksk_words);
    or_keygen(&op, 2021, olwe.data(), otlwe.data(), obk.data(), oksk.data());
    check(cemu_export_keys(sk, ck, lwe.data(), tlwe.data(), bk.data(), ksk.data()) == CEMU_OK, "export");
    check(lwe == olwe && tlwe == otlwe, "secret keys equal the oracle's");
    check(bk == obk, "bootstrapping key (recombined from its int8 limbs) equals the oracle's");
    check(ksk == oksk, "key-switching key equals the oracle's");

    // encryption, decryption, phase
    const int64_t B = 100;
    std::vector<uint8_t> bits(B), dec(B);
    for (int64_t i = 0; i < B; ++i) bits[(size_t)i] = (uint8_t)((i * 7 + 3) % 5 < 2);
    std::vector<uint32_t> ct((size_t)B * n1), oct((size_t)B * n1);
    check(cemu_encrypt(sk, bits.data(), B, 5, 1000, ct.data()) == CEMU_OK, "encrypt");
    or_encrypt_bits(&op, olwe.data(), 5, 1000, bits.data(), B, oct.data());
    check(ct == oct, "encryptions equal the oracle's");
    check(cemu_decrypt(sk, ct.data(), B, dec.data()) == CEMU_OK && dec == bits, "decrypt");
    std::vector<uint32_t> ph((size_t)B);
    check(cemu_phase(sk, 0, ct.data(), B, ph.data()) == CEMU_OK, "phase");
    bool ok = true;
    for (int64_t i = 0; i < B; ++i) ok &= ph[(size_t)i] == or_lwe_phase(n, olwe.data(), &ct[(size_t)i * n1]);
    check(ok, "phases equal the oracle's");
    // a dimension-N sample: trivial (0, ..., 0, +-1/8)
    std::vector<uint32_t> ext((size_t)2 * N1, 0u);
    ext[(size_t)N] = 0x20000000u;
    ext[(size_t)N1 + N] = 0xE0000000u;
    check(cemu_decrypt_extracted(sk, ext.data(), 2, dec.data()) == CEMU_OK && dec[0] == 1 && dec[1] == 0,
          "decrypt extracted");
    check(cemu_phase(sk, 1, ext.data(), 2, ph.data()) == CEMU_OK && ph[0] == 0x20000000u, "phase extracted");

    // argument checks
    check(cemu_encrypt(sk, bits.data(), -1, 5, 0, ct.data()) != CEMU_OK, "negative count refused");
    check(cemu_encrypt(nullptr, bits.data(), 1, 5, 0, ct.data()) == CEMU_ERR_NULL, "null key refused");
    check(cemu_decrypt(sk, nullptr, 1, dec.data()) == CEMU_ERR_NULL, "null ciphertexts refused");
    check(std::strlen(cemu_last_error()) > 0, "error message kept");
    cemu_params q;
    check(cemu_secret_params(sk, &q) == CEMU_OK && q.n == p.n && q.N == p.N, "secret parameters");
    check(cemu_cloud_params(ck, &q) == CEMU_OK && q.t == p.t, "cloud parameters");

    cemu_free_secret_key(sk);
    cemu_free_cloud_key(ck);
    std::printf("sanitized host run: %d failed checks\n", failures);
    return failures;
}
