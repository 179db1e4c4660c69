// Internal declarations shared by the host part (cemu_host.cpp) and the
// device part (cemu_device.hip) of libcemu. Not part of the public ABI.
#pragma once

#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/cemu.h"

struct cemu_secret_key {
    cemu_params p;
    std::vector<int32_t> lwe_key;   // [n]
    std::vector<int32_t> tlwe_key;  // [N]
};

// Device-resident cloud key plus per-key scratch workspaces.
struct cemu_cloud_key {
    cemu_params p;
    int device = -1;
    int num_cus = 0;   // compute units of that device (0: unknown)
    // Bootstrapping key, int8-limb layout. For step i, digit row r = c*l + j,
    // output component q and limb kappa, 2N bytes R with
    //   R[u] = limb_kappa( E[2N-1-u] ),  E[t] = BK[t-N] (t >= N), -BK[t] (t < N),
    // so that the negacyclic Toeplitz entry T[m][k] = BK*(X^k) at row m equals
    // R[N-1-m+k]. Layout [n][2l][2][4][2N] bytes.
    uint8_t *d_bk8 = nullptr;
    // Key-switching key, canonical layout [N][t][2^basebit][n+1] words.
    uint32_t *d_ksk = nullptr;
    // The same key as int8 limbs in MFMA B-operand order (see cemu_ks.hip),
    // present when the parameters allow the MFMA key switch (t = 8).
    uint8_t *d_ksk_mfma = nullptr;
    // Bootstrapping key in the FFT form (built at key generation, N = 1024): for step i and
    // row r, component q, the twisted spectrum of the centred key polynomial,
    // [n][2l][2][N/2] complex doubles stored as (re, im).
    double *d_bkfft = nullptr;
    // Scratch, grown on demand.
    uint16_t *d_bars = nullptr;  // [cap][n+1] mod-switched lincomb outputs
    int64_t bars_cap = 0;
    uint32_t *d_ext = nullptr;   // [cap][N+1] extracted samples
    int64_t ext_cap = 0;
    std::mutex mu;
    cemu_tuning tuning = {8, 8, 16, {0, 0, 0, 0, 0}};
    // Kernel timing (cemu_profile_enable): (kind, start, stop) event triples.
    mutable bool profiling = false;
    struct ProfileRec {
        int kind;
        void *start;
        void *stop;
    };
    mutable std::vector<ProfileRec> prof;
};

namespace cemu {

// Thread-local error reporting (cemu_host.cpp).
int fail(int code, const std::string &msg);
void clear_error();

// Parameter validation shared by host and device parts.
int check_params(const cemu_params *p);

// Kernel timing around one launch (cemu_device.hip). prof_begin returns an
// opaque start event or nullptr when profiling is off.
void *prof_begin(const cemu_cloud_key *ck, void *stream);
void prof_end(const cemu_cloud_key *ck, int kind, void *stream, void *start);

// Device-side helpers (cemu_device.hip).
int upload_cloud_key(cemu_cloud_key *ck, const std::vector<uint8_t> &bk8, const std::vector<uint32_t> &ksk,
                     const std::vector<uint8_t> &ksk_mfma);

// Key-switching key in MFMA fragment order (cemu_ks.hip).
bool ks_mfma_supported(const cemu_params &p);
size_t ks_mfma_bytes(const cemu_params &p);
int ks_mfma_ntiles(const cemu_params &p);
void ks_mfma_arrange(const cemu_params &p, const uint32_t *ksk, uint8_t *wf, int kappa, int ntile);
int download_bk8(const cemu_cloud_key *ck, std::vector<uint8_t> &bk8);
int download_ksk(const cemu_cloud_key *ck, std::vector<uint32_t> &ksk);
void release_cloud_key(cemu_cloud_key *ck);

}  // namespace cemu
