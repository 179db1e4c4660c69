// Key switching N -> n for a batch, as an int8 MFMA contraction (gfx950).
//
// For gate g with extracted sample (a'_0..a'_{N-1}, b'), key switching
// subtracts the key row KS[i][j][d] for every nonzero digit d = d_{g,i,j} of
// the rounded a'_i (unsigned base 4, t = 8 digits, most significant first):
//   out_g = (0, ..., 0, b'_g) - sum_{i,j} KS[i][j][d_{g,i,j}].
// With the one-hot matrix O[g][(i,j,v)] = [d_{g,i,j} = v] and the key rows as
// a matrix W[(i,j,v)][u] (rows with v = 0 set to zero) this is the product
// C = O * W over K = 4 N t, followed by out = (0, b') - C. A batch reads the
// 84 MB key once per 64-gate tile instead of once per gate, so the step is
// bound by the contraction, not by HBM. The key words are split into four
// signed 8-bit limbs (exact modulo 2^32) and recombined by Horner's rule in
// the int32 accumulators, as in the blind rotation.
//
// One wave per workgroup computes a 64-gate x 64-column tile: 4 x 4 MFMA
// tiles of v_mfma_i32_16x16x64_i8. Narrow batches (few tiles) also split the
// K range over grid.z: each split Horner-combines the four limb products of
// its K range (the recombination is linear), and the splits are summed into
// an output pre-set to (0, b') with 32-bit integer atomics, which wrap exactly
// like the single-pass sum and give the same result in any order. The one-hot A operand is generated in
// registers from the rounded a'_i (one u32 per lane per M-tile and K-tile);
// the B operand (key limbs) is pre-arranged at key generation in exactly the
// per-lane order of the MFMA B operand, so each fragment load is one
// coalesced 1 KiB wave read.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "cemu_kernels.h"

namespace cemu {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef unsigned u4 __attribute__((ext_vector_type(4)));

template <int B, int E, class F>
__device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

constexpr int KS_T = 8;          // digits per coefficient (t)
constexpr int KS_MT = 4;         // 16-gate M-tiles per wave
constexpr int KS_NT = 4;         // 16-column N-tiles per wave

template <int N, bool SPLIT>
__global__ __launch_bounds__(64) void ks_mfma_kernel(const uint32_t *__restrict__ ext, const u4 *__restrict__ wf,
                                                     int32_t n, int32_t ntiles, int64_t B,
                                                     const int32_t *__restrict__ io, uint32_t *__restrict__ out)
{
    constexpr int KT = N * KS_T * 4 / 64;   // 64-wide K-tiles
    const int lane = threadIdx.x;
    const int r = lane & 15, g4 = lane >> 4;
    const int64_t gbase = (int64_t)blockIdx.x * (16 * KS_MT);
    const int cb = blockIdx.y;                // 64-column block
    const int jb = 4 * (g4 & 1);              // first digit index of this lane's 4 dwords
    const int ihalf = g4 >> 1;                // which of the tile's two coefficients

    // Row pointers of this lane's 4 gates (clamped; dummy gates contribute 0).
    const uint32_t *erow[KS_MT];
    bool glive[KS_MT];
    static_for<0, KS_MT>([&](auto mI) {
        constexpr int mt = decltype(mI)::value;
        const int64_t g = gbase + 16 * mt + r;
        glive[mt] = g < B;
        erow[mt] = ext + (glive[mt] ? g : 0) * (N + 1);
    });

    v4i acc[KS_MT][KS_NT];
    static_for<0, KS_MT>([&](auto mI) {
        static_for<0, KS_NT>([&](auto nI) { acc[decltype(mI)::value][decltype(nI)::value] = v4i{0, 0, 0, 0}; });
    });

    const u4 *wbase = wf + (size_t)(cb * KS_NT) * KT * 64 + lane;   // + ((kappa*ntiles + nt)*KT + kt)*64
    const int kt0 = SPLIT ? (int)(blockIdx.z * (unsigned)KT / gridDim.z) : 0;
    const int kt1 = SPLIT ? (int)((blockIdx.z + 1) * (unsigned)KT / gridDim.z) : KT;

#pragma unroll 1
    for (int kappa = 3; kappa >= 0; --kappa) {
        if (kappa != 3) {
            static_for<0, KS_MT>([&](auto mI) {
                static_for<0, KS_NT>([&](auto nI) { acc[decltype(mI)::value][decltype(nI)::value] <<= 8; });
            });
        }
        const u4 *wk = wbase + (size_t)kappa * ntiles * KT * 64;
        // prefetch K-tile 0
        uint32_t xa[KS_MT];
        u4 wb[KS_NT];
        static_for<0, KS_MT>([&](auto mI) { xa[decltype(mI)::value] = erow[decltype(mI)::value][2 * kt0 + ihalf]; });
        static_for<0, KS_NT>([&](auto nI) { wb[decltype(nI)::value] = wk[((size_t)decltype(nI)::value * KT + kt0) * 64]; });
#pragma unroll 2
        for (int kt = kt0; kt < kt1; ++kt) {
            const int ktn = kt + 1 < kt1 ? kt + 1 : kt;
            uint32_t xn[KS_MT];
            u4 wn[KS_NT];
            static_for<0, KS_MT>([&](auto mI) { xn[decltype(mI)::value] = erow[decltype(mI)::value][2 * ktn + ihalf]; });
            static_for<0, KS_NT>([&](auto nI) {
                wn[decltype(nI)::value] = wk[((size_t)decltype(nI)::value * KT + ktn) * 64];
            });
            // one-hot digits: dword q <- byte d set, d = digit jb+q of round16(a')
            v4i af[KS_MT];
            static_for<0, KS_MT>([&](auto mI) {
                constexpr int mt = decltype(mI)::value;
                const uint32_t xb = glive[mt] ? ((xa[mt] + 0x8000u) >> 16) : 0u;
                uint32_t w[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const uint32_t d = (xb >> (14 - 2 * (jb + q))) & 3u;
                    w[q] = 1u << (8 * d);
                }
                af[mt] = v4i{(int)w[0], (int)w[1], (int)w[2], (int)w[3]};
            });
            static_for<0, KS_MT>([&](auto mI) {
                constexpr int mt = decltype(mI)::value;
                static_for<0, KS_NT>([&](auto nI) {
                    constexpr int nt = decltype(nI)::value;
                    const u4 bw = wb[nt];
                    acc[mt][nt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(af[mt], v4i{(int)bw.x, (int)bw.y, (int)bw.z, (int)bw.w},
                                                                        acc[mt][nt], 0, 0, 0);
                });
            });
            static_for<0, KS_MT>([&](auto mI) { xa[decltype(mI)::value] = xn[decltype(mI)::value]; });
            static_for<0, KS_NT>([&](auto nI) { wb[decltype(nI)::value] = wn[decltype(nI)::value]; });
        }
    }

    // out = (0, b') - C; lane holds rows 4*(lane>>4)+i, column lane&15 of each tile.
    static_for<0, KS_MT>([&](auto mI) {
        constexpr int mt = decltype(mI)::value;
        static_for<0, KS_NT>([&](auto nI) {
            constexpr int nt = decltype(nI)::value;
            const int col = cb * 64 + nt * 16 + r;
            if (col <= n) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int64_t g = gbase + 16 * mt + 4 * g4 + i;
                    if (g < B) {
                        const uint32_t v = 0u - (uint32_t)acc[mt][nt][i];
                        const int64_t orow = io ? (int64_t)io[g] : g;
                        uint32_t *o = out + orow * (int64_t)(n + 1) + col;
                        if constexpr (SPLIT) atomicAdd(o, v);
                        else *o = col == n ? v + ext[g * (N + 1) + N] : v;
                    }
                }
            }
        });
    });
}

// Output rows of a split-K key switch start as (0, ..., 0, b').
template <int N>
__global__ __launch_bounds__(256) void ks_init_kernel(const uint32_t *__restrict__ ext, int32_t n, int64_t B,
                                                      const int32_t *__restrict__ io, uint32_t *__restrict__ out)
{
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= B * (int64_t)(n + 1)) return;
    const int64_t g = k / (n + 1);
    const int col = (int)(k - g * (n + 1));
    const int64_t orow = io ? (int64_t)io[g] : g;
    out[orow * (int64_t)(n + 1) + col] = col == n ? ext[g * (N + 1) + N] : 0u;
}

}  // namespace

bool ks_mfma_supported(const cemu_params &p) { return p.t == KS_T && p.basebit == 2; }

size_t ks_mfma_bytes(const cemu_params &p)
{
    const size_t ntiles = (size_t)((p.n + 1 + 63) / 64) * 4;
    return (size_t)4 * ntiles * ((size_t)p.N * KS_T * 4 / 64) * 64 * 16;
}

// Host-side arrangement of the key-switching key into MFMA B fragments:
// [kappa][ntile16][ktile][lane][16 bytes], byte e of lane (col = lane&15,
// kgroup = lane>>4) of K-tile kt = limb kappa of W[k][16*ntile + col],
// k = 64 kt + 16 kgroup + e = (i*t + j)*4 + v. Fills the (kappa, ntile) slab.
void ks_mfma_arrange(const cemu_params &p, const uint32_t *ksk, uint8_t *wf, int kappa, int nt)
{
    const int n = p.n, N = p.N, t = p.t;
    const int ntiles = ((n + 1 + 63) / 64) * 4;
    const int KT = N * t * 4 / 64;
    size_t o = ((size_t)kappa * ntiles + nt) * (size_t)KT * 64 * 16;
    for (int kt = 0; kt < KT; ++kt)
        for (int lane = 0; lane < 64; ++lane)
            for (int e = 0; e < 16; ++e) {
                const int col = 16 * nt + (lane & 15);
                const int k = 64 * kt + 16 * (lane >> 4) + e;
                const int v = k & 3, ij = k >> 2, i = ij / t, j = ij % t;
                uint32_t val = 0;
                if (v != 0 && col <= n) val = ksk[(((size_t)i * t + j) * 4 + v) * (size_t)(n + 1) + col];
                // signed balanced limb kappa: peel kappa+1 limbs off the bottom
                uint32_t y = val;
                int8_t s = 0;
                for (int kk = 0; kk <= kappa; ++kk) {
                    s = (int8_t)(uint8_t)(y & 0xFFu);
                    y = (y - (uint32_t)(int32_t)s) >> 8;
                }
                wf[o++] = (uint8_t)s;
            }
}

int ks_mfma_ntiles(const cemu_params &p) { return ((p.n + 1 + 63) / 64) * 4; }

int launch_ks_mfma(const cemu_cloud_key *ck, const uint32_t *ext, const int32_t *io, uint32_t *out, int64_t B,
                   hipStream_t s)
{
    const int n = ck->p.n, N = ck->p.N;
    const int ntiles = ((n + 1 + 63) / 64) * 4;
    const int64_t gblocks = (B + 16 * KS_MT - 1) / (16 * KS_MT);
    const int64_t tiles = gblocks * (ntiles / KS_NT);
    // split the K range when the tiles alone leave the SIMDs short of waves
    // (one wave per workgroup): aim at about 2048 workgroups, at least 16
    // K-tiles per split. A 4096-gate batch (640 tiles) then runs 2 splits:
    // 0.60 ms against 0.83 ms unsplit and 0.65 ms with 4 splits (MI355X).
    const int KT = N * KS_T * 4 / 64;
    int splits = 1;
    while (tiles * splits * 2 <= 2048 && KT / (splits * 2) >= 16) splits *= 2;
    const dim3 grid((unsigned)gblocks, (unsigned)(ntiles / KS_NT), (unsigned)splits);
    const u4 *wf = reinterpret_cast<const u4 *>(ck->d_ksk_mfma);
    if (splits > 1) {
        const int64_t cells = B * (int64_t)(n + 1);
        const unsigned ib = (unsigned)((cells + 255) / 256);
        if (N == 1024) hipLaunchKernelGGL(ks_init_kernel<1024>, dim3(ib), dim3(256), 0, s, ext, n, B, io, out);
        else hipLaunchKernelGGL(ks_init_kernel<512>, dim3(ib), dim3(256), 0, s, ext, n, B, io, out);
    }
    if (N == 1024) {
        if (splits > 1) hipLaunchKernelGGL((ks_mfma_kernel<1024, true>), grid, dim3(64), 0, s, ext, wf, n, ntiles, B, io, out);
        else hipLaunchKernelGGL((ks_mfma_kernel<1024, false>), grid, dim3(64), 0, s, ext, wf, n, ntiles, B, io, out);
    } else {
        if (splits > 1) hipLaunchKernelGGL((ks_mfma_kernel<512, true>), grid, dim3(64), 0, s, ext, wf, n, ntiles, B, io, out);
        else hipLaunchKernelGGL((ks_mfma_kernel<512, false>), grid, dim3(64), 0, s, ext, wf, n, ntiles, B, io, out);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(CEMU_ERR_HIP, std::string("ks_mfma_kernel launch: ") + hipGetErrorString(e));
    return CEMU_OK;
}

}  // namespace cemu
