// Device part of libcemu for gfx950 (MI355X): key upload, the gate
// linear-combination + modulus-switch kernel, the two halves of the
// homomorphic MUX (its lincomb over 2B gates and the combine of the two
// extracted samples), circuit levels that mix gates and MUXes in one
// blind-rotation launch, the blind-rotation kernels (int8-MFMA form in
// cemu_br_int8.hip, FFT64 form in cemu_br_fft.hip), the key-switching
// kernels (MFMA form in cemu_ks.hip, VALU form here), the unbootstrapped
// NOT / COPY / CONSTANT kernels, and the device entry points of the C ABI.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>

#include "cemu_internal.h"
#include "cemu_kernels.h"

namespace cemu {

namespace {

std::string hip_msg(const char *what, hipError_t e)
{
    return std::string(what) + ": " + hipGetErrorString(e);
}

// Element-wise kernels walk their index range with a grid stride and their
// launches cap the grid: a dispatch counts its work-items in 32 bits, so one
// thread per element would limit a batch to 2^32 / (n + 1) gates. The cap
// (2^24 threads) is far above what the GPU holds resident.
constexpr int kElemThreads = 256;
constexpr int64_t kElemMaxBlocks = 1 << 16;

inline dim3 elem_grid(int64_t total)
{
    const int64_t b = (total + kElemThreads - 1) / kElemThreads;
    return dim3((unsigned)(b < kElemMaxBlocks ? b : kElemMaxBlocks));
}

#define ELEM_LOOP(idx, total)                                                                   \
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < (total);            \
         idx += (int64_t)gridDim.x * blockDim.x)

#define CEMU_HIP(call)                                                   \
    do {                                                                 \
        hipError_t e_ = (call);                                          \
        if (e_ != hipSuccess) return fail(CEMU_ERR_HIP, hip_msg(#call, e_)); \
    } while (0)

// Gate constants: (kappa, w1, w2) with c = (0,...,0,kappa) + w1*c1 + w2*c2.
// Encoding +-1/8 for bits; the gate set of Table "TFHEbenchmark".
__constant__ uint32_t c_gate_kappa[CEMU_NUM_GATE_OPS] = {
    0x20000000u, 0xE0000000u, 0x20000000u, 0x40000000u, 0xC0000000u,
    0xE0000000u, 0xE0000000u, 0xE0000000u, 0x20000000u, 0x20000000u};
__constant__ int32_t c_gate_w1[CEMU_NUM_GATE_OPS] = {-1, 1, 1, 2, -2, -1, -1, 1, -1, 1};
__constant__ int32_t c_gate_w2[CEMU_NUM_GATE_OPS] = {-1, 1, 1, 2, -2, -1, 1, -1, 1, -1};

// K1: gate linear combination fused with the modulus switch to Z/2N.
// One element per (gate, coefficient); bars is [B][n+1] u16 row-major.
__global__ void lincomb_modswitch_kernel(const uint8_t *__restrict__ ops, const uint32_t *__restrict__ pool,
                                         const int32_t *__restrict__ ia, const int32_t *__restrict__ ib,
                                         int32_t n, int32_t log2_2n, int64_t B, uint16_t *__restrict__ bars)
{
    const int64_t row = n + 1;
    // nearest integer to x * 2N / 2^32, mod 2N (the shift drops the wrap)
    const uint32_t half = 1u << (31 - log2_2n);
    ELEM_LOOP(idx, B * row) {
        const int64_t g = idx / row;
        const int32_t u = (int32_t)(idx - g * row);
        uint32_t op = ops[g];
        if (op >= CEMU_NUM_GATE_OPS) op = 0;
        const uint32_t x1 = pool[(int64_t)ia[g] * row + u];
        const uint32_t x2 = pool[(int64_t)ib[g] * row + u];
        uint32_t x = (uint32_t)c_gate_w1[op] * x1 + (uint32_t)c_gate_w2[op] * x2;
        if (u == n) x += c_gate_kappa[op];
        bars[idx] = (uint16_t)((x + half) >> (32 - log2_2n));
    }
}

// Multiplexer, first half: the two gates AND(s, a) and ANDNY(s, b) of every
// MUX g as one batch of 2B gates (g and B + g), lincomb and modulus switch
// exactly as lincomb_modswitch_kernel.
__global__ void mux_lincomb_kernel(const uint32_t *__restrict__ pool, const int32_t *__restrict__ is,
                                   const int32_t *__restrict__ ia, const int32_t *__restrict__ ib, int32_t n,
                                   int32_t log2_2n, int64_t B, uint16_t *__restrict__ bars)
{
    const int64_t row = n + 1;
    const uint32_t half = 1u << (31 - log2_2n);
    ELEM_LOOP(idx, 2 * B * row) {
        const int64_t g2 = idx / row;
        const int32_t u = (int32_t)(idx - g2 * row);
        const bool second = g2 >= B;
        const int64_t g = second ? g2 - B : g2;
        const int op = second ? CEMU_ANDNY : CEMU_AND;
        const uint32_t x1 = pool[(int64_t)is[g] * row + u];
        const uint32_t x2 = pool[(int64_t)(second ? ib[g] : ia[g]) * row + u];
        uint32_t x = (uint32_t)c_gate_w1[op] * x1 + (uint32_t)c_gate_w2[op] * x2;
        if (u == n) x += c_gate_kappa[op];
        bars[idx] = (uint16_t)((x + half) >> (32 - log2_2n));
    }
}

// Multiplexer, second half: ext[g] += ext[B + g] + (0, ..., 0, 1/8). Both
// extracted samples encrypt -1/8 except the one of the selected input when
// it is true, so the sum encrypts +-1/8 for the selected bit.
__global__ void mux_combine_kernel(uint32_t *__restrict__ ext, int32_t N, int64_t B)
{
    const int64_t row = N + 1;
    ELEM_LOOP(idx, B * row) {
        const int64_t j = idx - (idx / row) * row;
        ext[idx] += ext[idx + B * row] + (j == N ? 0x20000000u : 0u);
    }
}

// K3: key switching N -> n. A workgroup takes KS_G samples; thread t owns
// output columns t, t+256, t+512 for all of them. The rounded inputs are
// staged in LDS; each key row is read once per workgroup and applied to the
// KS_G samples from registers.
constexpr int KS_G = 16;
constexpr int KS_THREADS = 256;
constexpr int KS_COLS = 3;   // 3 * 256 >= n + 1 for n <= 767

template <int N>
__global__ __launch_bounds__(KS_THREADS) void key_switch_kernel(const uint32_t *__restrict__ ext,
                                                                const uint32_t *__restrict__ ksk, int32_t n,
                                                                int32_t t, int64_t B, const int32_t *__restrict__ io,
                                                                uint32_t *__restrict__ out)
{
    __shared__ uint32_t xr[KS_G][N];
    __shared__ uint32_t bprime[KS_G];
    const int tid = threadIdx.x;
    const int64_t g0 = (int64_t)blockIdx.x * KS_G;
    const int prec = 2 * t;                       // basebit = 2
    const uint32_t round = prec >= 32 ? 0u : (1u << (31 - prec));
    for (int e = tid; e < KS_G * N; e += KS_THREADS) {
        const int g = e / N, i = e - g * N;
        uint32_t v = 0;
        if (g0 + g < B) {
            const uint32_t a = ext[(g0 + g) * (N + 1) + i];
            v = prec >= 32 ? a : ((a + round) >> (32 - prec));
        }
        xr[g][i] = v;
    }
    if (tid < KS_G) bprime[tid] = (g0 + tid < B) ? ext[(g0 + tid) * (N + 1) + N] : 0u;
    __syncthreads();

    const int64_t rowlen = n + 1;
    uint32_t acc[KS_G][KS_COLS];
#pragma unroll
    for (int g = 0; g < KS_G; ++g)
#pragma unroll
        for (int c = 0; c < KS_COLS; ++c) acc[g][c] = 0u;
    int col[KS_COLS];
    bool ok[KS_COLS];
#pragma unroll
    for (int c = 0; c < KS_COLS; ++c) {
        col[c] = tid + c * KS_THREADS;
        ok[c] = col[c] <= n;
        if (!ok[c]) col[c] = n;  // keep loads in bounds; result discarded
    }
    for (int i = 0; i < N; ++i) {
        for (int j = 0; j < t; ++j) {
            const uint32_t *rows = ksk + ((int64_t)i * t + j) * 4 * rowlen;
            uint32_t r1[KS_COLS], r2[KS_COLS], r3[KS_COLS];
#pragma unroll
            for (int c = 0; c < KS_COLS; ++c) {
                r1[c] = rows[rowlen + col[c]];
                r2[c] = rows[2 * rowlen + col[c]];
                r3[c] = rows[3 * rowlen + col[c]];
            }
            const int sh = prec - 2 * (j + 1);
#pragma unroll
            for (int g = 0; g < KS_G; ++g) {
                const uint32_t d = (xr[g][i] >> sh) & 3u;
#pragma unroll
                for (int c = 0; c < KS_COLS; ++c) {
                    const uint32_t v = d == 1u ? r1[c] : (d == 2u ? r2[c] : (d == 3u ? r3[c] : 0u));
                    acc[g][c] -= v;
                }
            }
        }
    }
#pragma unroll
    for (int g = 0; g < KS_G; ++g) {
        if (g0 + g >= B) break;
        const int64_t orow = io ? (int64_t)io[g0 + g] : g0 + g;
#pragma unroll
        for (int c = 0; c < KS_COLS; ++c) {
            if (!ok[c]) continue;
            uint32_t v = acc[g][c];
            if (col[c] == n) v += bprime[g];
            out[orow * rowlen + col[c]] = v;
        }
    }
}

__global__ void lwe_not_kernel(int32_t n, const uint32_t *__restrict__ in, const int32_t *__restrict__ src,
                               uint32_t *__restrict__ out, const int32_t *__restrict__ dst, int64_t count)
{
    const int64_t row = n + 1;
    ELEM_LOOP(idx, count * row) {
        const int64_t e = idx / row, u = idx - e * row;
        out[(int64_t)dst[e] * row + u] = 0u - in[(int64_t)src[e] * row + u];
    }
}

__global__ void lwe_copy_kernel(int32_t n, const uint32_t *__restrict__ in, const int32_t *__restrict__ src,
                                uint32_t *__restrict__ out, const int32_t *__restrict__ dst, int64_t count)
{
    const int64_t row = n + 1;
    ELEM_LOOP(idx, count * row) {
        const int64_t e = idx / row, u = idx - e * row;
        out[(int64_t)dst[e] * row + u] = in[(int64_t)src[e] * row + u];
    }
}

__global__ void lwe_constant_kernel(int32_t n, const uint8_t *__restrict__ bits, uint32_t *__restrict__ out,
                                    const int32_t *__restrict__ dst, int64_t count)
{
    const int64_t row = n + 1;
    ELEM_LOOP(idx, count * row) {
        const int64_t e = idx / row, u = idx - e * row;
        out[(int64_t)dst[e] * row + u] = u == n ? (bits[e] ? 0x20000000u : 0xE0000000u) : 0u;
    }
}

inline bool misaligned(const void *p) { return ((uintptr_t)p & 3u) != 0; }

// Largest batch an entry point accepts: keeps every element count and byte
// size computed from it far from int64 / size_t overflow (real batches are
// bounded much earlier by device memory).
constexpr int64_t kMaxBatch = (int64_t)1 << 40;

// CEMU_KS_VALU=1 selects the VALU key-switching kernel (for comparison).
bool ks_valu_forced()
{
    static const bool f = [] {
        const char *e = std::getenv("CEMU_KS_VALU");
        return e && e[0] == '1';
    }();
    return f;
}


// Fixed scratch of cemu_bootstrap_gates_noalloc, for callers that cannot
// allocate: the rescaled masks (u16 [B][n+1], n + 1 <= 768) and then the
// extracted samples (u32 [B][N+1], N <= 1024) of up to CEMU_NOALLOC_MAX_GATES
// gates, 22 MiB, present on every device the library runs on until the
// process ends. Host code must never pass the array's name to a kernel: on
// the host it is a stand-in, not a device address. The address of each
// device's copy comes from hipGetSymbolAddress with that device current.
constexpr size_t kNoallocBarsBytes = (size_t)CEMU_NOALLOC_MAX_GATES * (CEMU_MAX_KEY_N + 1) * sizeof(uint16_t);
constexpr size_t kNoallocExtBytes = (size_t)CEMU_NOALLOC_MAX_GATES * (1024 + 1) * sizeof(uint32_t);
static_assert(kNoallocBarsBytes % 256 == 0, "the sample region starts 256-byte aligned");
__device__ __align__(256) uint8_t scratch[kNoallocBarsBytes + kNoallocExtBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint8_t *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device dev, which must be current: looked
// up once per device (at key generation) and cached.
int noalloc_scratch(int dev, uint8_t **out)
{
    if (dev < 0 || dev >= kMaxDevices) return fail(CEMU_ERR_PARAM, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return fail(CEMU_ERR_HIP, hip_msg("hipGetSymbolAddress (scratch)", e));
        g_scratch_ptr[dev] = static_cast<uint8_t *>(p);
    }
    *out = g_scratch_ptr[dev];
    return CEMU_OK;
}

int ensure_workspace(cemu_cloud_key *ck, int64_t B, bool need_ext)
{
    const int32_t n = ck->p.n, N = ck->p.N;
    if (ck->bars_cap < B) {
        if (ck->d_bars) CEMU_HIP(hipFree(ck->d_bars));
        ck->d_bars = nullptr;
        ck->bars_cap = 0;
        if (hipMalloc(&ck->d_bars, (size_t)B * (n + 1) * sizeof(uint16_t)) != hipSuccess)
            return fail(CEMU_ERR_OOM, "device workspace allocation failed");
        ck->bars_cap = B;
    }
    if (need_ext && ck->ext_cap < B) {
        if (ck->d_ext) CEMU_HIP(hipFree(ck->d_ext));
        ck->d_ext = nullptr;
        ck->ext_cap = 0;
        if (hipMalloc(&ck->d_ext, (size_t)B * (N + 1) * sizeof(uint32_t)) != hipSuccess)
            return fail(CEMU_ERR_OOM, "device workspace allocation failed");
        ck->ext_cap = B;
    }
    return CEMU_OK;
}

// A launch that failed after prof_begin: drop its start event, report.
int launch_failed(void *ev, const char *what, hipError_t e)
{
    if (ev) (void)hipEventDestroy((hipEvent_t)ev);
    return fail(CEMU_ERR_HIP, hip_msg(what, e));
}

int log2_of(int v)
{
    int r = 0;
    while ((1 << r) < v) ++r;
    return r;
}

int launch_lincomb(const cemu_cloud_key *ck, const uint8_t *ops, const uint32_t *pool, const int32_t *ia,
                   const int32_t *ib, int64_t B, uint16_t *bars, hipStream_t s)
{
    const int32_t n = ck->p.n;
    void *ev = prof_begin(ck, s);
    hipLaunchKernelGGL(lincomb_modswitch_kernel, elem_grid(B * (n + 1)), dim3(kElemThreads), 0, s, ops, pool, ia, ib,
                       n, log2_of(2 * ck->p.N), B, bars);
    if (const hipError_t e = hipGetLastError(); e != hipSuccess) return launch_failed(ev, "lincomb launch", e);
    prof_end(ck, 0, s, ev);
    return CEMU_OK;
}

int launch_key_switch(const cemu_cloud_key *ck, const uint32_t *ext, const int32_t *io, uint32_t *out, int64_t B,
                      hipStream_t s)
{
    const int32_t n = ck->p.n, N = ck->p.N, t = ck->p.t;
    if (n + 1 > KS_COLS * KS_THREADS) return fail(CEMU_ERR_UNSUPPORTED, "key switch supports n <= 767");
    void *ev = prof_begin(ck, s);
    if (ck->d_ksk_mfma && ks_mfma_supported(ck->p) && !ks_valu_forced()) {
        const int rc = launch_ks_mfma(ck, ext, io, out, B, s);
        if (rc == CEMU_OK) prof_end(ck, 3, s, ev);
        else if (ev) (void)hipEventDestroy((hipEvent_t)ev);
        return rc;
    }
    const int64_t blocks = (B + KS_G - 1) / KS_G;
    if (N == 1024)
        hipLaunchKernelGGL(key_switch_kernel<1024>, dim3((unsigned)blocks), dim3(KS_THREADS), 0, s, ext, ck->d_ksk, n,
                           t, B, io, out);
    else
        hipLaunchKernelGGL(key_switch_kernel<512>, dim3((unsigned)blocks), dim3(KS_THREADS), 0, s, ext, ck->d_ksk, n,
                           t, B, io, out);
    if (const hipError_t e = hipGetLastError(); e != hipSuccess) return launch_failed(ev, "key switch launch", e);
    prof_end(ck, 3, s, ev);
    return CEMU_OK;
}

// The blind-rotation launch for B rotations fits one dispatch (checked
// before anything is allocated or launched).
int check_br_batch(const cemu_cloud_key *ck, int form, int64_t B)
{
    return form == CEMU_FORM_INT8 ? br_int8_batch_ok(ck, B) : br_fft_batch_ok(ck, B);
}

int check_device(const cemu_cloud_key *ck)
{
    int dev = -1;
    CEMU_HIP(hipGetDevice(&dev));
    if (dev != ck->device) return fail(CEMU_ERR_PARAM, "current HIP device differs from the cloud key's device");
    return CEMU_OK;
}

// Blind rotation + extraction of the B gates whose rescaled masks are in bars.
int run_br(cemu_cloud_key *ck, int form, const uint16_t *bars, uint32_t *ext_out, int64_t B, hipStream_t s)
{
    int rc;
    void *ev = prof_begin(ck, s);
    if (form == CEMU_FORM_INT8) rc = launch_br_int8(ck, bars, B, ext_out, s);
    else if (form == CEMU_FORM_FFT64) rc = launch_br_fft(ck, bars, B, ext_out, s);
    else rc = fail(CEMU_ERR_PARAM, "unknown product form");
    if (rc == CEMU_OK) prof_end(ck, form == CEMU_FORM_INT8 ? 1 : 2, s, ev);
    else if (ev) (void)hipEventDestroy((hipEvent_t)ev);
    return rc;
}

// Lincomb + blind rotation + extraction into ext_out ([B][N+1]); bars is
// the [B][n+1] workspace of the rescaled masks.
int run_blind_rotate(cemu_cloud_key *ck, int form, const uint8_t *ops, const uint32_t *pool, const int32_t *ia,
                     const int32_t *ib, uint16_t *bars, uint32_t *ext_out, int64_t B, hipStream_t s)
{
    int rc = launch_lincomb(ck, ops, pool, ia, ib, B, bars, s);
    if (rc) return rc;
    return run_br(ck, form, bars, ext_out, B, s);
}

// G gates and M multiplexers through one blind-rotation launch and one key
// switch. Workspace rows: [0, G) the gates, [G, G + M) the AND(s, a) halves
// and [G + M, G + 2M) the ANDNY(s, b) halves of the multiplexers; after the
// combine, rows [0, G + M) are the samples to key-switch, in output order.
int run_level(cemu_cloud_key *ck, int form, const uint32_t *pool, const uint8_t *ops, const int32_t *ia,
              const int32_t *ib, int64_t G, const int32_t *ms, const int32_t *ma, const int32_t *mb, int64_t M,
              const int32_t *io, uint32_t *pool_out, hipStream_t s)
{
    const int32_t n = ck->p.n, N = ck->p.N;
    int rc;
    if (G > 0 && (rc = launch_lincomb(ck, ops, pool, ia, ib, G, ck->d_bars, s))) return rc;
    if (M > 0) {
        void *ev = prof_begin(ck, s);
        hipLaunchKernelGGL(mux_lincomb_kernel, elem_grid(2 * M * (n + 1)), dim3(kElemThreads), 0, s, pool, ms, ma, mb,
                           n, log2_of(2 * N), M, ck->d_bars + G * (n + 1));
        if (const hipError_t e = hipGetLastError(); e != hipSuccess) return launch_failed(ev, "MUX lincomb launch", e);
        prof_end(ck, 0, s, ev);
    }
    rc = run_br(ck, form, ck->d_bars, ck->d_ext, G + 2 * M, s);
    if (rc) return rc;
    if (M > 0) {
        hipLaunchKernelGGL(mux_combine_kernel, elem_grid(M * (N + 1)), dim3(kElemThreads), 0, s,
                           ck->d_ext + G * (N + 1), N, M);
        CEMU_HIP(hipGetLastError());
    }
    return launch_key_switch(ck, ck->d_ext, io, pool_out, G + M, s);
}

}  // namespace

void *prof_begin(const cemu_cloud_key *ck, void *stream)
{
    if (!ck->profiling) return nullptr;
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    if (hipEventRecord(e, (hipStream_t)stream) != hipSuccess) {
        (void)hipEventDestroy(e);
        return nullptr;
    }
    return (void *)e;
}

void prof_end(const cemu_cloud_key *ck, int kind, void *stream, void *start)
{
    if (!start) return;
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess || hipEventRecord(e, (hipStream_t)stream) != hipSuccess) {
        if (e) (void)hipEventDestroy(e);
        (void)hipEventDestroy((hipEvent_t)start);
        return;
    }
    ck->prof.push_back({kind, start, (void *)e});
}

int upload_cloud_key(cemu_cloud_key *ck, const std::vector<uint8_t> &bk8, const std::vector<uint32_t> &ksk,
                     const std::vector<uint8_t> &ksk_mfma)
{
    CEMU_HIP(hipGetDevice(&ck->device));
    if (hipDeviceGetAttribute(&ck->num_cus, hipDeviceAttributeMultiprocessorCount, ck->device) != hipSuccess)
        ck->num_cus = 0;
    if (hipMalloc(&ck->d_bk8, bk8.size()) != hipSuccess) return fail(CEMU_ERR_OOM, "device allocation (BK) failed");
    if (hipMalloc(&ck->d_ksk, ksk.size() * sizeof(uint32_t)) != hipSuccess) {
        release_cloud_key(ck);
        return fail(CEMU_ERR_OOM, "device allocation (KSK) failed");
    }
    if (!ksk_mfma.empty() && hipMalloc(&ck->d_ksk_mfma, ksk_mfma.size()) != hipSuccess) {
        release_cloud_key(ck);
        return fail(CEMU_ERR_OOM, "device allocation (KSK, MFMA layout) failed");
    }
    hipError_t e1 = hipMemcpy(ck->d_bk8, bk8.data(), bk8.size(), hipMemcpyHostToDevice);
    hipError_t e2 = hipMemcpy(ck->d_ksk, ksk.data(), ksk.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
    hipError_t e3 = ksk_mfma.empty() ? hipSuccess
                                     : hipMemcpy(ck->d_ksk_mfma, ksk_mfma.data(), ksk_mfma.size(), hipMemcpyHostToDevice);
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
        release_cloud_key(ck);
        return fail(CEMU_ERR_HIP, hip_msg("hipMemcpy (key upload)", e1 != hipSuccess ? e1 : (e2 != hipSuccess ? e2 : e3)));
    }
    // the FFT form of the key, and this device's address of the fixed
    // scratch, so that later gate calls need no set-up
    int rc = CEMU_OK;
    if (ck->p.N == 1024) {
        rc = build_bk_fft(ck, nullptr);
        if (rc == CEMU_OK) {
            const hipError_t e = hipStreamSynchronize(nullptr);
            if (e != hipSuccess) rc = fail(CEMU_ERR_HIP, hip_msg("FFT key preparation", e));
        }
    }
    uint8_t *scr = nullptr;
    if (rc == CEMU_OK) rc = noalloc_scratch(ck->device, &scr);
    if (rc != CEMU_OK) release_cloud_key(ck);
    return rc;
}

int download_bk8(const cemu_cloud_key *ck, std::vector<uint8_t> &bk8)
{
    const cemu_params &p = ck->p;
    bk8.resize((size_t)p.n * 2 * p.l * 2 * 4 * 2 * p.N);
    CEMU_HIP(hipMemcpy(bk8.data(), ck->d_bk8, bk8.size(), hipMemcpyDeviceToHost));
    return CEMU_OK;
}

int download_ksk(const cemu_cloud_key *ck, std::vector<uint32_t> &ksk)
{
    const cemu_params &p = ck->p;
    ksk.resize((size_t)p.N * p.t * (1 << p.basebit) * (p.n + 1));
    CEMU_HIP(hipMemcpy(ksk.data(), ck->d_ksk, ksk.size() * sizeof(uint32_t), hipMemcpyDeviceToHost));
    return CEMU_OK;
}

void release_cloud_key(cemu_cloud_key *ck)
{
    if (ck->d_bk8) (void)hipFree(ck->d_bk8);
    if (ck->d_ksk) (void)hipFree(ck->d_ksk);
    if (ck->d_ksk_mfma) (void)hipFree(ck->d_ksk_mfma);
    if (ck->d_bkfft) (void)hipFree(ck->d_bkfft);
    if (ck->d_bars) (void)hipFree(ck->d_bars);
    if (ck->d_ext) (void)hipFree(ck->d_ext);
    ck->d_bk8 = nullptr;
    ck->d_ksk = nullptr;
    ck->d_ksk_mfma = nullptr;
    ck->d_bkfft = nullptr;
    ck->d_bars = nullptr;
    ck->d_ext = nullptr;
    ck->bars_cap = ck->ext_cap = 0;
}

}  // namespace cemu

using namespace cemu;

extern "C" {

int cemu_bootstrap_gates(const cemu_cloud_key *ckc, int form, const uint8_t *ops, const uint32_t *pool_in,
                         const int32_t *ia, const int32_t *ib, const int32_t *io, uint32_t *pool_out, int64_t B,
                         void *hip_stream)
{
    clear_error();
    if (!ckc) return fail(CEMU_ERR_NULL, "cloud key is NULL");
    if (B < 0) return fail(CEMU_ERR_RANGE, "B < 0");
    if (form != CEMU_FORM_INT8 && form != CEMU_FORM_FFT64) return fail(CEMU_ERR_PARAM, "unknown product form");
    if (B == 0) return CEMU_OK;
    if (B > kMaxBatch) return fail(CEMU_ERR_RANGE, "batch too large");
    if (!ops || !pool_in || !ia || !ib || !pool_out) return fail(CEMU_ERR_NULL, "NULL device buffer");
    if (misaligned(pool_in) || misaligned(ia) || misaligned(ib) || misaligned(pool_out) || (io && misaligned(io)))
        return fail(CEMU_ERR_ALIGN, "device buffers must be 4-byte aligned");
    cemu_cloud_key *ck = const_cast<cemu_cloud_key *>(ckc);
    std::lock_guard<std::mutex> lock(ck->mu);
    int rc = check_device(ck);
    if (rc) return rc;
    if ((rc = check_br_batch(ck, form, B))) return rc;
    rc = ensure_workspace(ck, B, true);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)hip_stream;
    rc = run_blind_rotate(ck, form, ops, pool_in, ia, ib, ck->d_bars, ck->d_ext, B, s);
    if (rc) return rc;
    return launch_key_switch(ck, ck->d_ext, io, pool_out, B, s);
}

int cemu_bootstrap_gates_noalloc(const cemu_cloud_key *ckc, int form, const uint8_t *ops, const uint32_t *pool_in,
                                 const int32_t *ia, const int32_t *ib, const int32_t *io, uint32_t *pool_out,
                                 int64_t B, void *hip_stream)
{
    clear_error();
    if (!ckc) return fail(CEMU_ERR_NULL, "cloud key is NULL");
    if (B < 0) return fail(CEMU_ERR_RANGE, "B < 0");
    if (form != CEMU_FORM_INT8 && form != CEMU_FORM_FFT64) return fail(CEMU_ERR_PARAM, "unknown product form");
    if (B == 0) return CEMU_OK;
    if (B > CEMU_NOALLOC_MAX_GATES)
        return fail(CEMU_ERR_RANGE, "batch larger than the fixed scratch of cemu_bootstrap_gates_noalloc "
                                    "(CEMU_NOALLOC_MAX_GATES = 4096 gates)");
    if (!ops || !pool_in || !ia || !ib || !pool_out) return fail(CEMU_ERR_NULL, "NULL device buffer");
    if (misaligned(pool_in) || misaligned(ia) || misaligned(ib) || misaligned(pool_out) || (io && misaligned(io)))
        return fail(CEMU_ERR_ALIGN, "device buffers must be 4-byte aligned");
    cemu_cloud_key *ck = const_cast<cemu_cloud_key *>(ckc);
    std::lock_guard<std::mutex> lock(ck->mu);
    int rc = check_device(ck);
    if (rc) return rc;
    if ((rc = check_br_batch(ck, form, B))) return rc;
    if (form == CEMU_FORM_FFT64 && !ck->d_bkfft)
        return fail(CEMU_ERR_UNSUPPORTED, "the FFT64 form needs N = 1024 (its key is built at key generation)");
    uint8_t *scr = nullptr;
    if ((rc = noalloc_scratch(ck->device, &scr))) return rc;
    // the masks, then the extracted samples: every word of both is written
    // before it is read, so nothing needs clearing between calls
    uint16_t *bars = reinterpret_cast<uint16_t *>(scr);
    uint32_t *ext = reinterpret_cast<uint32_t *>(scr + kNoallocBarsBytes);
    // kernel timing creates events; this entry point records none
    const bool profiling = ck->profiling;
    ck->profiling = false;
    hipStream_t s = (hipStream_t)hip_stream;
    rc = run_blind_rotate(ck, form, ops, pool_in, ia, ib, bars, ext, B, s);
    if (rc == CEMU_OK) rc = launch_key_switch(ck, ext, io, pool_out, B, s);
    ck->profiling = profiling;
    return rc;
}

int cemu_mux(const cemu_cloud_key *ckc, int form, const uint32_t *pool_in, const int32_t *is, const int32_t *ia,
             const int32_t *ib, const int32_t *io, uint32_t *pool_out, int64_t B, void *hip_stream)
{
    clear_error();
    if (!ckc) return fail(CEMU_ERR_NULL, "cloud key is NULL");
    if (B < 0) return fail(CEMU_ERR_RANGE, "B < 0");
    if (form != CEMU_FORM_INT8 && form != CEMU_FORM_FFT64) return fail(CEMU_ERR_PARAM, "unknown product form");
    if (B == 0) return CEMU_OK;
    if (B > kMaxBatch) return fail(CEMU_ERR_RANGE, "batch too large");
    if (!pool_in || !is || !ia || !ib || !pool_out) return fail(CEMU_ERR_NULL, "NULL device buffer");
    if (misaligned(pool_in) || misaligned(is) || misaligned(ia) || misaligned(ib) || misaligned(pool_out) ||
        (io && misaligned(io)))
        return fail(CEMU_ERR_ALIGN, "device buffers must be 4-byte aligned");
    cemu_cloud_key *ck = const_cast<cemu_cloud_key *>(ckc);
    std::lock_guard<std::mutex> lock(ck->mu);
    int rc = check_device(ck);
    if (rc) return rc;
    if ((rc = check_br_batch(ck, form, 2 * B))) return rc;
    rc = ensure_workspace(ck, 2 * B, true);
    if (rc) return rc;
    return run_level(ck, form, pool_in, nullptr, nullptr, nullptr, 0, is, ia, ib, B, io, pool_out,
                     (hipStream_t)hip_stream);
}

int cemu_bootstrap_level(const cemu_cloud_key *ckc, int form, const uint32_t *pool_in, const uint8_t *ops,
                         const int32_t *ia, const int32_t *ib, int64_t G, const int32_t *ms, const int32_t *ma,
                         const int32_t *mb, int64_t M, const int32_t *io, uint32_t *pool_out, void *hip_stream)
{
    clear_error();
    if (!ckc) return fail(CEMU_ERR_NULL, "cloud key is NULL");
    if (G < 0 || M < 0) return fail(CEMU_ERR_RANGE, "G < 0 or M < 0");
    if (form != CEMU_FORM_INT8 && form != CEMU_FORM_FFT64) return fail(CEMU_ERR_PARAM, "unknown product form");
    if (G == 0 && M == 0) return CEMU_OK;
    if (G > kMaxBatch || M > kMaxBatch) return fail(CEMU_ERR_RANGE, "batch too large");
    if (!pool_in || !pool_out || (G > 0 && (!ops || !ia || !ib)) || (M > 0 && (!ms || !ma || !mb)))
        return fail(CEMU_ERR_NULL, "NULL device buffer");
    if (misaligned(pool_in) || misaligned(pool_out) || (io && misaligned(io)) ||
        (G > 0 && (misaligned(ia) || misaligned(ib))) || (M > 0 && (misaligned(ms) || misaligned(ma) || misaligned(mb))))
        return fail(CEMU_ERR_ALIGN, "device buffers must be 4-byte aligned");
    cemu_cloud_key *ck = const_cast<cemu_cloud_key *>(ckc);
    std::lock_guard<std::mutex> lock(ck->mu);
    int rc = check_device(ck);
    if (rc) return rc;
    if ((rc = check_br_batch(ck, form, G + 2 * M))) return rc;
    rc = ensure_workspace(ck, G + 2 * M, true);
    if (rc) return rc;
    return run_level(ck, form, pool_in, ops, ia, ib, G, ms, ma, mb, M, io, pool_out, (hipStream_t)hip_stream);
}

int cemu_blind_rotate_extract(const cemu_cloud_key *ckc, int form, const uint8_t *ops, const uint32_t *pool_in,
                              const int32_t *ia, const int32_t *ib, uint32_t *out_N, int64_t B, void *hip_stream)
{
    clear_error();
    if (!ckc) return fail(CEMU_ERR_NULL, "cloud key is NULL");
    if (B < 0) return fail(CEMU_ERR_RANGE, "B < 0");
    if (form != CEMU_FORM_INT8 && form != CEMU_FORM_FFT64) return fail(CEMU_ERR_PARAM, "unknown product form");
    if (B == 0) return CEMU_OK;
    if (B > kMaxBatch) return fail(CEMU_ERR_RANGE, "batch too large");
    if (!ops || !pool_in || !ia || !ib || !out_N) return fail(CEMU_ERR_NULL, "NULL device buffer");
    if (misaligned(pool_in) || misaligned(ia) || misaligned(ib) || misaligned(out_N))
        return fail(CEMU_ERR_ALIGN, "device buffers must be 4-byte aligned");
    cemu_cloud_key *ck = const_cast<cemu_cloud_key *>(ckc);
    std::lock_guard<std::mutex> lock(ck->mu);
    int rc = check_device(ck);
    if (rc) return rc;
    if ((rc = check_br_batch(ck, form, B))) return rc;
    rc = ensure_workspace(ck, B, false);
    if (rc) return rc;
    return run_blind_rotate(ck, form, ops, pool_in, ia, ib, ck->d_bars, out_N, B, (hipStream_t)hip_stream);
}

int cemu_key_switch(const cemu_cloud_key *ck, const uint32_t *in_N, uint32_t *out_n, int64_t B, void *hip_stream)
{
    clear_error();
    if (!ck) return fail(CEMU_ERR_NULL, "cloud key is NULL");
    if (B < 0) return fail(CEMU_ERR_RANGE, "B < 0");
    if (B == 0) return CEMU_OK;
    if (B > kMaxBatch) return fail(CEMU_ERR_RANGE, "batch too large");
    if (!in_N || !out_n) return fail(CEMU_ERR_NULL, "NULL device buffer");
    if (misaligned(in_N) || misaligned(out_n)) return fail(CEMU_ERR_ALIGN, "device buffers must be 4-byte aligned");
    std::lock_guard<std::mutex> lock(const_cast<cemu_cloud_key *>(ck)->mu);
    int rc = check_device(ck);
    if (rc) return rc;
    return launch_key_switch(ck, in_N, nullptr, out_n, B, (hipStream_t)hip_stream);
}

int cemu_get_tuning(const cemu_cloud_key *ck, cemu_tuning *t)
{
    clear_error();
    if (!ck || !t) return fail(CEMU_ERR_NULL, "NULL argument");
    *t = ck->tuning;
    return CEMU_OK;
}

int cemu_set_tuning(cemu_cloud_key *ck, const cemu_tuning *t)
{
    clear_error();
    if (!ck || !t) return fail(CEMU_ERR_NULL, "NULL argument");
    if (t->int8_waves != 4 && t->int8_waves != 8) return fail(CEMU_ERR_PARAM, "int8_waves must be 4 or 8");
    if (t->fft_gates_per_wg != 1 && t->fft_gates_per_wg != 4 && t->fft_gates_per_wg != 8)
        return fail(CEMU_ERR_PARAM, "fft_gates_per_wg must be 1, 4 or 8");
    if (t->int8_gates_per_wg != 0 && t->int8_gates_per_wg != 1 && t->int8_gates_per_wg != 16)
        return fail(CEMU_ERR_PARAM, "int8_gates_per_wg must be 1 or 16 (0 selects 16)");
    std::lock_guard<std::mutex> lock(ck->mu);
    ck->tuning = *t;
    if (ck->tuning.int8_gates_per_wg == 0) ck->tuning.int8_gates_per_wg = 16;
    return CEMU_OK;
}

int cemu_profile_enable(cemu_cloud_key *ck, int enable)
{
    clear_error();
    if (!ck) return fail(CEMU_ERR_NULL, "cloud key is NULL");
    std::lock_guard<std::mutex> lock(ck->mu);
    ck->profiling = enable != 0;
    return CEMU_OK;
}

int cemu_profile_read(cemu_cloud_key *ck, double *ms, int64_t *launches)
{
    clear_error();
    if (!ck) return fail(CEMU_ERR_NULL, "cloud key is NULL");
    std::lock_guard<std::mutex> lock(ck->mu);
    double sum[CEMU_PROFILE_KINDS] = {0, 0, 0, 0};
    int64_t cnt[CEMU_PROFILE_KINDS] = {0, 0, 0, 0};
    int rc = CEMU_OK;
    for (auto &r : ck->prof) {
        float t = 0.f;
        hipError_t e = hipEventSynchronize((hipEvent_t)r.stop);
        if (e == hipSuccess) e = hipEventElapsedTime(&t, (hipEvent_t)r.start, (hipEvent_t)r.stop);
        if (e != hipSuccess && rc == CEMU_OK) rc = fail(CEMU_ERR_HIP, hip_msg("profile event", e));
        if (r.kind >= 0 && r.kind < CEMU_PROFILE_KINDS) {
            sum[r.kind] += t;
            cnt[r.kind] += 1;
        }
        (void)hipEventDestroy((hipEvent_t)r.start);
        (void)hipEventDestroy((hipEvent_t)r.stop);
    }
    ck->prof.clear();
    for (int k = 0; k < CEMU_PROFILE_KINDS; ++k) {
        if (ms) ms[k] = sum[k];
        if (launches) launches[k] = cnt[k];
    }
    return rc;
}

static int launch_rowwise(int which, int32_t n, const uint32_t *in, const int32_t *src, const uint8_t *bits,
                          uint32_t *out, const int32_t *dst, int64_t count, void *hip_stream)
{
    clear_error();
    if (count < 0) return fail(CEMU_ERR_RANGE, "count < 0");
    if (n < 1 || n > CEMU_MAX_LWE_N) return fail(CEMU_ERR_PARAM, "n must be in [1, CEMU_MAX_LWE_N]");
    if (count == 0) return CEMU_OK;
    if (count > kMaxBatch) return fail(CEMU_ERR_RANGE, "count too large");
    if (!out || !dst || (which < 2 && (!in || !src)) || (which == 2 && !bits))
        return fail(CEMU_ERR_NULL, "NULL device buffer");
    const dim3 grid = elem_grid(count * (n + 1)), block(kElemThreads);
    hipStream_t s = (hipStream_t)hip_stream;
    if (which == 0) hipLaunchKernelGGL(lwe_not_kernel, grid, block, 0, s, n, in, src, out, dst, count);
    else if (which == 1) hipLaunchKernelGGL(lwe_copy_kernel, grid, block, 0, s, n, in, src, out, dst, count);
    else hipLaunchKernelGGL(lwe_constant_kernel, grid, block, 0, s, n, bits, out, dst, count);
    CEMU_HIP(hipGetLastError());
    return CEMU_OK;
}

int cemu_lwe_not(int32_t n, const uint32_t *pool_in, const int32_t *src, uint32_t *pool_out, const int32_t *dst,
                 int64_t count, void *hip_stream)
{
    return launch_rowwise(0, n, pool_in, src, nullptr, pool_out, dst, count, hip_stream);
}

int cemu_lwe_copy(int32_t n, const uint32_t *pool_in, const int32_t *src, uint32_t *pool_out, const int32_t *dst,
                  int64_t count, void *hip_stream)
{
    return launch_rowwise(1, n, pool_in, src, nullptr, pool_out, dst, count, hip_stream);
}

int cemu_lwe_constant(int32_t n, const uint8_t *bits, uint32_t *pool_out, const int32_t *dst, int64_t count,
                      void *hip_stream)
{
    return launch_rowwise(2, n, nullptr, nullptr, bits, pool_out, dst, count, hip_stream);
}

}  // extern "C"
