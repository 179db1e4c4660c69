// Blind rotation with exact int8-MFMA negacyclic products (gfx950).
//
// One workgroup owns BR_G = 16 gates for all n CMux steps; their
// accumulators ACC = (A, B) stay in LDS. Step i computes
//   ACC += BK_i [external product] (X^{abar_i} ACC - ACC)
// as an integer GEMM per digit row p = c*l + j (c: accumulator component,
// j: gadget level) and output component q:
//   Delta_q[m][g] = sum_p sum_k T_{p,q}[m][k] * d_p[k][g]     (mod 2^32)
// where T_{p,q} is the negacyclic Toeplitz matrix of the key polynomial
// BK_i[p][q] and d_p are the signed 7-bit digits of gate g. The Torus32 key
// coefficients are split into four signed 8-bit limbs (exact mod 2^32), each
// limb product runs on v_mfma_i32_16x16x64_i8 (A = Toeplitz rows, B = digits
// of the 16 gates), and the limbs are recombined inside the int32
// accumulator by Horner's rule: acc = ((C3*2^8 + C2)*2^8 + C1)*2^8 + C0,
// which is exact because int32 MFMA accumulation wraps modulo 2^32.
//
// The Toeplitz A operand is never materialised. For output rows m and
// columns k, T[m][k] = R[N-1-m+k] with R the reversed, sign-extended limb
// sequence of the key (see cemu_internal.h), so a lane's 16 A bytes are 16
// consecutive bytes of R. A tile of T depends only on the difference of its
// row and column offsets, so each generated fragment is reused for every
// (M-tile, K-tile) pair on that diagonal.
//
// Per digit row p the workgroup first computes the digits of all 16 gates
// into LDS (each digit once), then every wave loads its B operand from there.
// The first half of the waves computes output component A, the second half
// B, and each keeps the step's running sum in registers until the
// accumulators are updated. Two tilings: br_int8_res_kernel (8 waves, the
// default) gives each wave the rows of one residue class mod 4, which makes
// every fragment four whole dwords (see there); br_int8_kernel (the 4-wave
// shape) gives each wave a block of consecutive rows, whose fragments start
// at any byte and are fetched as 5 dwords and shifted with v_alignbyte.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "cemu_kernels.h"

namespace cemu {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef unsigned u4 __attribute__((ext_vector_type(4)));

// Compile-time loop: f(std::integral_constant<int, I>) for I in [B, E). Used
// wherever a register array is indexed, so that every index is a constant
// and the arrays stay in registers.
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

constexpr int BR_G = 16;    // gates per workgroup = MFMA N dimension
constexpr int BR_ROWS = 6;  // (k+1) * l digit rows, k = 1, l = 3

template <int N, int WAVES>
struct BrShape {
    static constexpr int THREADS = 64 * WAVES;
    static constexpr int PARTS = WAVES / 2;                     // waves per output component
    static constexpr int RW = N / PARTS;                        // output rows per wave
    static constexpr int MT = RW / 16;                          // 16-row M-tiles per wave
    static constexpr int KT = N / 64;                           // 64-wide K-tiles per digit row
    static constexpr int RB = 2 * N;                            // bytes of one limb sequence R
    static constexpr int STAGE_BYTES = 2 * 4 * RB;              // R for one digit row: (q, limb)
    static constexpr int NDELTA = (MT - 1) + 4 * (KT - 1) + 1;  // distinct fragments per block
    static constexpr int PRE = STAGE_BYTES / (THREADS * 16);    // u4 per thread per stage
    static constexpr int CHUNKS = BR_G * N / 16;                // 16-digit chunks per digit row
    static constexpr int CPT = CHUNKS / THREADS;                // chunks per thread
    static_assert(PRE >= 1 && CPT >= 1 && MT >= 1, "shape");
};

// OFF = sum_{j=1..3} (Bg/2) 2^(32-7j) + 2^(32-21-1): adding it turns the
// signed rounded digits into plain bit fields: d_j = ((x+OFF) >> (32-7j)) & 127) - 64.
constexpr uint32_t kDigitOffset = 0x81020400u;

// Accumulator word k of gate g lives at g*N + (k ^ acc_swz(g)). The XOR keeps
// 4-word groups contiguous and spreads the 16 gates over distinct LDS banks
// for the column-wise (MFMA output) and row-wise (digit) access patterns.
__device__ __forceinline__ uint32_t acc_swz(int g) { return (uint32_t)(((g & 3) << 4) | ((g >> 2) << 2)); }

// Digit chunk ch (digits of coefficients 16ch..16ch+15) of gate g lives at
// byte g*N + 16*(ch ^ g): the 16 lanes that read one K-group hit 16 banks.
__device__ __forceinline__ uint32_t dig_off(int N, int g, int ch) { return (uint32_t)(g * N + 16 * (ch ^ (g & 15))); }

// acc[a] += T_tile(a, b) * D_tile(b) for all (a, b), one limb; a fragment is
// generated once per diagonal delta = 4b - a and reused for every pair on it.
template <int N, int WAVES>
__device__ __forceinline__ void mfma_block(const uint32_t *__restrict__ pr, uint32_t shift,
                                           v4i (&acc)[BrShape<N, WAVES>::MT], const v4i (&bf)[BrShape<N, WAVES>::KT])
{
    using S = BrShape<N, WAVES>;
    // Software pipeline: the dwords of fragment d+1 are requested before the
    // MFMAs of fragment d are issued; sched_barrier keeps that order.
    uint32_t w0 = pr[0], w1 = pr[1], w2 = pr[2], w3 = pr[3], w4 = pr[4];
    static_for<0, S::NDELTA>([&](auto dI) {
        constexpr int di = decltype(dI)::value;
        const v4i fr = v4i{(int)__builtin_amdgcn_alignbyte(w1, w0, shift), (int)__builtin_amdgcn_alignbyte(w2, w1, shift),
                           (int)__builtin_amdgcn_alignbyte(w3, w2, shift), (int)__builtin_amdgcn_alignbyte(w4, w3, shift)};
        uint32_t n1 = 0, n2 = 0, n3 = 0, n4 = 0;
        if constexpr (di + 1 < S::NDELTA) {
            n1 = pr[4 * di + 5];
            n2 = pr[4 * di + 6];
            n3 = pr[4 * di + 7];
            n4 = pr[4 * di + 8];
        }
        static_for<0, S::KT>([&](auto bI) {
            constexpr int b = decltype(bI)::value;
            constexpr int a = 4 * b - (di - (S::MT - 1));
            if constexpr (a >= 0 && a < S::MT) acc[a] = __builtin_amdgcn_mfma_i32_16x16x64_i8(fr, bf[b], acc[a], 0, 0, 0);
        });
        w0 = w4;
        w1 = n1;
        w2 = n2;
        w3 = n3;
        w4 = n4;
        __builtin_amdgcn_sched_barrier(0);
    });
}

template <int N, int WAVES>
__global__ __launch_bounds__(64 * WAVES, 1) void br_int8_kernel(const uint8_t *__restrict__ bk8,
                                                                const uint16_t *__restrict__ bars, int32_t n,
                                                                int64_t B, uint32_t *__restrict__ ext)
{
    using S = BrShape<N, WAVES>;
    __shared__ __attribute__((aligned(16))) uint32_t acc_s[2][BR_G * N];
    __shared__ __attribute__((aligned(16))) uint8_t dig[BR_G * N];
    __shared__ __attribute__((aligned(16))) uint32_t rst[S::STAGE_BYTES / 4];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int q = wave / S::PARTS, part = wave - q * S::PARTS;
    const int gl = lane & 15, g4 = lane >> 4;
    const int64_t g0 = (int64_t)blockIdx.x * BR_G;
    const int64_t barrow = (int64_t)n + 1;
    const bool live = g0 + gl < B;
    const uint16_t *mybars = bars + (g0 + gl) * barrow;
    const uint32_t myswz = acc_swz(gl);

    // ACC = (0, X^{-bbar} v), v = (1/8) sum_j X^j.
    for (int e = tid; e < BR_G * N; e += S::THREADS) {
        const int g = e / N, m = e - (e / N) * N;
        const uint32_t bb = (g0 + g < B) ? (uint32_t)bars[(g0 + g) * barrow + n] : 0u;
        const uint32_t tt = ((uint32_t)m + bb) & (uint32_t)(2 * N - 1);
        const uint32_t ph = (uint32_t)(g * N) + ((uint32_t)m ^ acc_swz(g));
        acc_s[0][ph] = 0u;
        acc_s[1][ph] = tt < (uint32_t)N ? 0x20000000u : 0xE0000000u;
    }

    // Lane's A-fragment source: s0 = N-1 - part*RW - r + 16*kgroup - 16*(MT-1) >= 0.
    const int s0 = (N - 1) - part * S::RW - gl + 16 * g4 - 16 * (S::MT - 1);
    const uint32_t frag_shift = (uint32_t)(s0 & 3);
    const int frag_dw = s0 >> 2;

    // Register-staged prefetch of the next digit row's key limbs.
    u4 pre[S::PRE];
    {
        const u4 *src = reinterpret_cast<const u4 *>(bk8);
        static_for<0, S::PRE>([&](auto kI) { pre[decltype(kI)::value] = src[tid + decltype(kI)::value * S::THREADS]; });
    }

    uint32_t a_cur = live ? (uint32_t)mybars[0] : 0u;
    v4i total[S::MT];

    for (int i = 0; i < n; ++i) {
        const uint32_t a_next = (live && i + 1 < n) ? (uint32_t)mybars[i + 1] : 0u;
        static_for<0, S::MT>([&](auto tI) { total[decltype(tI)::value] = v4i{0, 0, 0, 0}; });

#pragma unroll 1
        for (int p = 0; p < BR_ROWS; ++p) {
            __syncthreads();  // previous digit row fully consumed; ACC updates visible
            {
                u4 *dst = reinterpret_cast<u4 *>(rst);
                static_for<0, S::PRE>([&](auto kI) { dst[tid + decltype(kI)::value * S::THREADS] = pre[decltype(kI)::value]; });
            }
            {
                // next (step, row); past the last step reload row 0 (unused)
                int ni = i, np = p + 1;
                if (np == BR_ROWS) {
                    np = 0;
                    ++ni;
                }
                if (ni >= n) ni = 0;
                const u4 *src = reinterpret_cast<const u4 *>(bk8 + ((size_t)ni * BR_ROWS + np) * S::STAGE_BYTES);
                static_for<0, S::PRE>([&](auto kI) { pre[decltype(kI)::value] = src[tid + decltype(kI)::value * S::THREADS]; });
            }
            // Digits of row p = (c, j) of X^a*ACC_c - ACC_c for all 16 gates:
            // thread handles chunks f = tid + r*THREADS, gate f&15 (= gl).
            {
                const int c = p / 3, j = p - (p / 3) * 3;
                const uint32_t sh = (uint32_t)(32 - 7 * (j + 1));
                const uint32_t *row = &acc_s[c][gl * N];
#pragma unroll 1
                for (int r = 0; r < S::CPT; ++r) {
                    const int ch = (tid + r * S::THREADS) >> 4;
                    const int k0 = 16 * ch;
                    uint32_t packed[4];
#pragma unroll
                    for (int d = 0; d < 4; ++d) {
                        const u4 uw = *reinterpret_cast<const u4 *>(row + ((uint32_t)(k0 + 4 * d) ^ myswz));
                        const uint32_t un[4] = {uw.x, uw.y, uw.z, uw.w};
                        uint32_t word = 0;
#pragma unroll
                        for (int e4 = 0; e4 < 4; ++e4) {
                            const uint32_t k = (uint32_t)(k0 + 4 * d + e4);
                            const uint32_t tt = (k - a_cur) & (uint32_t)(2 * N - 1);
                            uint32_t v = row[(tt & (uint32_t)(N - 1)) ^ myswz];
                            v = (tt & (uint32_t)N) ? 0u - v : v;
                            const uint32_t y = v - un[e4] + kDigitOffset;
                            word |= ((y >> sh) & 127u) << (8 * e4);
                        }
                        // bytes x in [0,128) hold digit + 64; (x + 64) ^ 0x80 = x - 64 mod 256, no carries
                        packed[d] = (word + 0x40404040u) ^ 0x80808080u;
                    }
                    *reinterpret_cast<u4 *>(dig + dig_off(N, gl, ch)) = u4{packed[0], packed[1], packed[2], packed[3]};
                }
            }
            __syncthreads();  // digits and key stage visible

            v4i bf[S::KT];
            static_for<0, S::KT>([&](auto bI) {
                constexpr int b = decltype(bI)::value;
                const u4 d4 = *reinterpret_cast<const u4 *>(dig + dig_off(N, gl, 4 * b + g4));
                bf[b] = v4i{(int)d4.x, (int)d4.y, (int)d4.z, (int)d4.w};
            });

            v4i acc[S::MT];
            static_for<0, S::MT>([&](auto tI) { acc[decltype(tI)::value] = v4i{0, 0, 0, 0}; });
            // Issue balance: with 8 waves, waves w and w + 4 share a SIMD and
            // do the same work; the arbiter issues the older one first, so the
            // younger raises its priority for the first three of the four limb
            // passes (88.6 against 89.7 ms per 4096 gates; two passes 89.0,
            // all four 91.1 against 91.8 on a slower box).
            if (WAVES == 8 && wave >= 4) __builtin_amdgcn_s_setprio(1);
#pragma unroll 1
            for (int kappa = 3; kappa >= 0; --kappa) {
                if (kappa == 0) __builtin_amdgcn_s_setprio(0);
                if (kappa != 3) static_for<0, S::MT>([&](auto tI) { acc[decltype(tI)::value] <<= 8; });
                const uint32_t *pr = rst + (q * 4 + kappa) * (S::RB / 4) + frag_dw;
                mfma_block<N, WAVES>(pr, frag_shift, acc, bf);
            }
            static_for<0, S::MT>([&](auto tI) { total[decltype(tI)::value] += acc[decltype(tI)::value]; });
        }
        __syncthreads();  // every wave has finished reading ACC for this step
        static_for<0, S::MT>([&](auto tI) {
            constexpr int t = decltype(tI)::value;
            const uint32_t m = (uint32_t)(part * S::RW + 16 * t + 4 * g4);
            u4 *ptr = reinterpret_cast<u4 *>(&acc_s[q][gl * N + (m ^ myswz)]);
            u4 v = *ptr;
            v.x += (uint32_t)total[t][0];
            v.y += (uint32_t)total[t][1];
            v.z += (uint32_t)total[t][2];
            v.w += (uint32_t)total[t][3];
            *ptr = v;
        });
        a_cur = a_next;
    }
    __syncthreads();

    // Sample extraction: a'_0 = A_0, a'_j = -A_{N-j}, b' = B_0.
    for (int e = tid; e < BR_G * (N + 1); e += S::THREADS) {
        const int g = e / (N + 1), jj = e - (e / (N + 1)) * (N + 1);
        if (g0 + g >= B) continue;
        const uint32_t base = (uint32_t)(g * N), sw = acc_swz(g);
        uint32_t v;
        if (jj == 0) v = acc_s[0][base + (0u ^ sw)];
        else if (jj == N) v = acc_s[1][base + (0u ^ sw)];
        else v = 0u - acc_s[0][base + ((uint32_t)(N - jj) ^ sw)];
        ext[(g0 + g) * (N + 1) + jj] = v;
    }
}

// Residue-class tiling of the 16-gate product (8 waves). Wave w computes
// output component q = w / 4 and, of it, the rows m = v (mod 4), v = w % 4:
// tile u is rows 64 u + v + 4 r', r' = 0..15, and the wave's K range is
// shifted by c = (v + 1) mod 4, i.e. K-tile b is columns 64 b + c .. + 63.
// A lane (row r', K-group g4) then needs the 16 bytes of R starting at
//   N - 1 - m + k = N - 4 r' + 16 g4 + 64 (b - u) - 4 [v = 3],
// a dword boundary, so a fragment is four whole dwords with no byte
// alignment; and it depends on b - u only, so one fragment serves every
// (u, b) pair on that diagonal: 256 MFMAs per 31 fragments (N = 1024)
// against 76 with blocks of consecutive rows. The columns shifted past N
// wrap around: column N + k' (k' < c = v + 1, so k' <= v <= m; for v = 3
// nothing wraps) meets R[2N - 1 - m + k'] = -T[m][k'], so it is fed the
// negated digit -d[k'] (digits are in [-64, 64), so their negations fit a
// signed byte).
//
// ACC row m of a gate is kept at the permuted position
//   P(m) = (m & ~15) | ((m & 3) << 2) | ((m >> 2) & 3)
// (then XOR-swizzled by gate as in br_int8_kernel), which puts the four rows
// 4 apart that one lane of an MFMA tile holds into one 16-byte group, and
// keeps each 16-coefficient digit chunk in four 16-byte groups.
template <int N>
struct ResShape {
    static constexpr int THREADS = 512;
    static constexpr int MT = N / 64;              // tiles per wave (64-row blocks of one component)
    static constexpr int KT = N / 64;              // 64-wide K-tiles
    static constexpr int DLO = -(MT - 1);          // lowest diagonal b - u
    static constexpr int NDELTA = KT + MT - 1;
    static constexpr int RB = 2 * N;
    static constexpr int STAGE_BYTES = 2 * 4 * RB;
    static constexpr int PRE = STAGE_BYTES / (THREADS * 16);
    static constexpr int CHUNKS = BR_G * N / 16;
    static constexpr int CPT = CHUNKS / THREADS;
    static_assert(MT >= 1 && PRE >= 1 && CPT >= 1, "shape");
};

__device__ __forceinline__ uint32_t res_perm(uint32_t m) { return (m & ~15u) | ((m & 3u) << 2) | ((m >> 2) & 3u); }

// Bytes of a packed word of signed digits, negated: with b = x ^ 0x80 = d + 128
// in [64, 191] per byte, ~b + 1 = 128 - d stays inside its byte.
__device__ __forceinline__ uint32_t neg_digits(uint32_t x) { return ((~(x ^ 0x80808080u)) + 0x01010101u) ^ 0x80808080u; }

// acc[u] += T_tile(u, b) * D_tile(b), one limb; pr points at the lane's first
// fragment (diagonal DLO), 16 dwords per diagonal. FRESH: acc holds nothing
// yet, so each tile's first product (b = 0, the first in diagonal order)
// starts from zero instead of reading acc.
template <int N, bool FRESH = false>
__device__ __forceinline__ void res_block(const uint32_t *__restrict__ pr, v4i (&acc)[ResShape<N>::MT],
                                          const v4i (&bf)[ResShape<N>::KT])
{
    using S = ResShape<N>;
    // Software pipeline: fragment di + 1 is requested before the MFMAs of
    // fragment di are issued; sched_barrier keeps that order.
    v4i fr = v4i{(int)pr[0], (int)pr[1], (int)pr[2], (int)pr[3]};
    static_for<0, S::NDELTA>([&](auto dI) {
        constexpr int di = decltype(dI)::value;
        v4i nx = fr;
        if constexpr (di + 1 < S::NDELTA)
            nx = v4i{(int)pr[16 * di + 16], (int)pr[16 * di + 17], (int)pr[16 * di + 18], (int)pr[16 * di + 19]};
        static_for<0, S::MT>([&](auto uI) {
            constexpr int u = decltype(uI)::value;
            constexpr int b = di + S::DLO + u;
            if constexpr (b >= 0 && b < S::KT)
                acc[u] = __builtin_amdgcn_mfma_i32_16x16x64_i8(fr, bf[b], (FRESH && b == 0) ? v4i{0, 0, 0, 0} : acc[u],
                                                               0, 0, 0);
        });
        fr = nx;
        __builtin_amdgcn_sched_barrier(0);
    });
}

template <int N>
__global__ __launch_bounds__(512, 1) void br_int8_res_kernel(const uint8_t *__restrict__ bk8,
                                                             const uint16_t *__restrict__ bars, int32_t n, int64_t B,
                                                             uint32_t *__restrict__ ext)
{
    using S = ResShape<N>;
    __shared__ __attribute__((aligned(16))) uint32_t acc_s[2][BR_G * N];
    __shared__ __attribute__((aligned(16))) uint8_t dig[BR_G * N];
    __shared__ __attribute__((aligned(16))) uint32_t rst[S::STAGE_BYTES / 4];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int q = wave >> 2, v = wave & 3;                        // output component, row residue
    const int gl = lane & 15, g4 = lane >> 4;
    const int c = (v + 1) & 3;                                     // K shift of this wave
    const int64_t g0 = (int64_t)blockIdx.x * BR_G;
    const int64_t barrow = (int64_t)n + 1;
    const bool live = g0 + gl < B;
    const uint16_t *mybars = bars + (g0 + gl) * barrow;
    const uint32_t myswz = acc_swz(gl);

    // ACC = (0, X^{-bbar} v), v = (1/8) sum_j X^j.
    for (int e = tid; e < BR_G * N; e += S::THREADS) {
        const int g = e / N, m = e - (e / N) * N;
        const uint32_t bb = (g0 + g < B) ? (uint32_t)bars[(g0 + g) * barrow + n] : 0u;
        const uint32_t tt = ((uint32_t)m + bb) & (uint32_t)(2 * N - 1);
        const uint32_t ph = (uint32_t)(g * N) + (res_perm((uint32_t)m) ^ acc_swz(g));
        acc_s[0][ph] = 0u;
        acc_s[1][ph] = tt < (uint32_t)N ? 0x20000000u : 0xE0000000u;
    }

    // The lane's first fragment: byte N - 4 r' + 16 g4 - 4 [v = 3] + 64 DLO >= 0
    // of R (a dword boundary), in the limb sequences of component q.
    const int frag_dw = (N - 4 * gl + 16 * g4 - (v == 3 ? 4 : 0) + 64 * S::DLO) / 4 + q * 4 * (S::RB / 4);

    // Register-staged prefetch of the next digit row's key limbs.
    u4 pre[S::PRE];
    {
        const u4 *src = reinterpret_cast<const u4 *>(bk8);
        static_for<0, S::PRE>([&](auto kI) { pre[decltype(kI)::value] = src[tid + decltype(kI)::value * S::THREADS]; });
    }

    uint32_t a_cur = live ? (uint32_t)mybars[0] : 0u;
    v4i total[S::MT];

    for (int i = 0; i < n; ++i) {
        const uint32_t a_next = (live && i + 1 < n) ? (uint32_t)mybars[i + 1] : 0u;
        static_for<0, S::MT>([&](auto tI) { total[decltype(tI)::value] = v4i{0, 0, 0, 0}; });

#pragma unroll 1
        for (int p = 0; p < BR_ROWS; ++p) {
            __syncthreads();  // previous digit row fully consumed; ACC updates visible
            {
                u4 *dst = reinterpret_cast<u4 *>(rst);
                static_for<0, S::PRE>([&](auto kI) { dst[tid + decltype(kI)::value * S::THREADS] = pre[decltype(kI)::value]; });
            }
            {
                // next (step, row); past the last step reload row 0 (unused)
                int ni = i, np = p + 1;
                if (np == BR_ROWS) {
                    np = 0;
                    ++ni;
                }
                if (ni >= n) ni = 0;
                const u4 *src = reinterpret_cast<const u4 *>(bk8 + ((size_t)ni * BR_ROWS + np) * S::STAGE_BYTES);
                static_for<0, S::PRE>([&](auto kI) { pre[decltype(kI)::value] = src[tid + decltype(kI)::value * S::THREADS]; });
            }
            // Digits of row p = (c, j) of X^a*ACC_c - ACC_c for all 16 gates:
            // thread handles chunks f = tid + r*THREADS, gate f&15 (= gl).
            {
                const int cc = p / 3, j = p - (p / 3) * 3;
                const uint32_t sh = (uint32_t)(32 - 7 * (j + 1));
                const uint32_t *row = &acc_s[cc][gl * N];
#pragma unroll 1
                for (int r = 0; r < S::CPT; ++r) {
                    const int ch = (tid + r * S::THREADS) >> 4;
                    const int k0 = 16 * ch;
                    // 16-byte group e4 of the chunk holds coefficients e4, 4 + e4, 8 + e4, 12 + e4
                    uint32_t packed[4] = {0u, 0u, 0u, 0u};
#pragma unroll
                    for (int e4 = 0; e4 < 4; ++e4) {
                        const u4 uw = *reinterpret_cast<const u4 *>(row + (((uint32_t)(k0 + 4 * e4)) ^ myswz));
                        const uint32_t un[4] = {uw.x, uw.y, uw.z, uw.w};
#pragma unroll
                        for (int d = 0; d < 4; ++d) {
                            const uint32_t k = (uint32_t)(k0 + 4 * d + e4);
                            const uint32_t tt = (k - a_cur) & (uint32_t)(2 * N - 1);
                            uint32_t vv = row[res_perm(tt & (uint32_t)(N - 1)) ^ myswz];
                            vv = (tt & (uint32_t)N) ? 0u - vv : vv;
                            const uint32_t y = vv - un[d] + kDigitOffset;
                            packed[d] |= ((y >> sh) & 127u) << (8 * e4);
                        }
                    }
                    // bytes x in [0,128) hold digit + 64; (x + 64) ^ 0x80 = x - 64 mod 256, no carries
#pragma unroll
                    for (int d = 0; d < 4; ++d) packed[d] = (packed[d] + 0x40404040u) ^ 0x80808080u;
                    *reinterpret_cast<u4 *>(dig + dig_off(N, gl, ch)) = u4{packed[0], packed[1], packed[2], packed[3]};
                }
            }
            __syncthreads();  // digits and key stage visible

            // B operand: bytes c .. c + 15 of chunks (4 b + g4, 4 b + g4 + 1) of
            // gate gl; past the last chunk the row wraps to chunk 0, negated.
            v4i bf[S::KT];
            static_for<0, S::KT>([&](auto bI) {
                constexpr int b = decltype(bI)::value;
                const int ch0 = 4 * b + g4;
                const u4 lo = *reinterpret_cast<const u4 *>(dig + dig_off(N, gl, ch0));
                u4 hi = *reinterpret_cast<const u4 *>(dig + dig_off(N, gl, (ch0 + 1) & (N / 16 - 1)));
                if constexpr (b == S::KT - 1) {
                    if (g4 == 3) hi = u4{neg_digits(hi.x), neg_digits(hi.y), neg_digits(hi.z), neg_digits(hi.w)};
                }
                const uint32_t s = (uint32_t)c;
                bf[b] = v4i{(int)__builtin_amdgcn_alignbyte(lo.y, lo.x, s), (int)__builtin_amdgcn_alignbyte(lo.z, lo.y, s),
                            (int)__builtin_amdgcn_alignbyte(lo.w, lo.z, s), (int)__builtin_amdgcn_alignbyte(hi.x, lo.w, s)};
            });

            // Horner over the limbs: acc = (C3 * 2^8 + C2) * 2^8 + C1, then the
            // last limb's products are accumulated straight onto
            // total + acc * 2^8. Issue balance: waves w and w + 4 share a SIMD
            // and do the same work; the arbiter issues the older one first, so
            // the younger raises its priority for the first three limb passes.
            v4i acc[S::MT];
            if (wave >= 4) __builtin_amdgcn_s_setprio(1);
            res_block<N, true>(rst + frag_dw + 3 * (S::RB / 4), acc, bf);
#pragma unroll 1
            for (int kappa = 2; kappa >= 1; --kappa) {
                static_for<0, S::MT>([&](auto tI) { acc[decltype(tI)::value] <<= 8; });
                res_block<N>(rst + frag_dw + kappa * (S::RB / 4), acc, bf);
            }
            __builtin_amdgcn_s_setprio(0);
            static_for<0, S::MT>([&](auto tI) {
                constexpr int t = decltype(tI)::value;
                total[t] += acc[t] << 8;
            });
            res_block<N>(rst + frag_dw, total, bf);
        }
        __syncthreads();  // every wave has finished reading ACC for this step
        // lane (gl, g4) of tile u holds rows 64 u + 16 g4 + 4 e + v, e = 0..3,
        // which P puts at 64 u + 16 g4 + 4 v + e; the swizzle touches bits 2..5
        // only, so the tiles of a lane are 64 u apart
        const uint32_t upd = (uint32_t)(gl * N) + ((uint32_t)(16 * g4 + 4 * v) ^ myswz);
        static_for<0, S::MT>([&](auto tI) {
            constexpr int u = decltype(tI)::value;
            u4 *ptr = reinterpret_cast<u4 *>(&acc_s[q][upd + 64 * u]);
            u4 w = *ptr;
            w.x += (uint32_t)total[u][0];
            w.y += (uint32_t)total[u][1];
            w.z += (uint32_t)total[u][2];
            w.w += (uint32_t)total[u][3];
            *ptr = w;
        });
        a_cur = a_next;
    }
    __syncthreads();

    // Sample extraction: a'_0 = A_0, a'_j = -A_{N-j}, b' = B_0.
    for (int e = tid; e < BR_G * (N + 1); e += S::THREADS) {
        const int g = e / (N + 1), jj = e - (e / (N + 1)) * (N + 1);
        if (g0 + g >= B) continue;
        const uint32_t base = (uint32_t)(g * N), sw = acc_swz(g);
        uint32_t val;
        if (jj == 0) val = acc_s[0][base + (res_perm(0u) ^ sw)];
        else if (jj == N) val = acc_s[1][base + (res_perm(0u) ^ sw)];
        else val = 0u - acc_s[0][base + (res_perm((uint32_t)(N - jj)) ^ sw)];
        ext[(g0 + g) * (N + 1) + jj] = val;
    }
}

// Latency kernel (narrow circuit levels): one gate per workgroup, so a level
// of G gates keeps G compute units busy instead of G / 16. With one gate the
// digits cannot fill the MFMA's 16 columns, so the roles are swapped: the A
// operand is the negacyclic Toeplitz matrix of the gate's own digit row,
//   T_p[m][k] = E_p[m - k],  E_p[s] = d_p[s] (s >= 0), -d_p[s + N] (s < 0),
// kept in LDS as X_p[v] = E_p[v - N], v in [0, 2N) (digits are int8, so the
// negated half is exact). X is stored four times, copy r shifted down by r
// bytes, so a lane whose 16-byte window starts at byte s reads four whole
// dwords from copy s & 3 and forms its fragment without byte alignment
// instructions.
//
// One level of the negacyclic half split: with H = N/2, T_p is the block
// matrix [[P, -Q], [Q, P]] of two H x H Toeplitz blocks, P[m][k] =
// E_p[m - k] and Q[m][k] = E_p[m - k + H] (the upper-right block is -Q
// because E_p[s - H] = -E_p[s + H] for the wrap). With the key split into
// halves k0 (coefficients < H) and k1, the product is
//   y0 = P k0 - Q k1,   y1 = Q k0 + P k1,
// two block products of half size, each against both key halves. The B
// operand holds the key limbs in all 16 columns: column n = 8 h + 4 q +
// kappa is limb kappa of half h of BK_i[p][q]. So one MFMA over a block
// serves both halves, and a digit row costs two H x H products (N^2 / 2
// multiply-adds in 16-column MFMAs) instead of one N x N product in which
// half of the columns would be zero.
//
// The limbs are recombined across the four lanes of a quad (shift by
// 8 kappa, then a reduce-scatter with two DPP exchanges that leaves each
// lane one full row) and each lane adds its row into ACC with an LDS integer
// atomic, negated for the -Q k1 term; the adds wrap modulo 2^32 like the sum
// itself, so their order does not matter and the result is bit-exact.
// Inside a lane's 16-byte group the k order is reversed in both operands
// (k = k0 + 16 g + 15 - t for byte t), which turns the key's reversed storage
// (BK[m] at byte N - 1 - m) into one aligned 16-byte load per K-tile and
// leaves X in natural order. Waves: component c (its 3 digit rows), block
// pr (P or Q), and for WAVES = 8 a half ks of the K-tiles of each row.
template <int N, int WAVES>
struct LatShape {
    static constexpr int THREADS = 64 * WAVES;
    static constexpr int KS = WAVES / 4;            // K-splits per (component, block)
    static constexpr int MT = N / 32;               // 16-row M-tiles per wave (the N/2 rows of a block)
    static constexpr int KT = N / 128 / KS;         // 64-wide K-tiles per wave and digit row (N/2 columns)
    static constexpr int NDELTA = MT + 4 * (KT - 1);
    static constexpr int XD = N / 2;                // dwords per extended digit row X_p
    static constexpr int XCOPY = BR_ROWS * XD + 8;  // dwords per shifted copy; +8 staggers the copies' banks
    static_assert(WAVES == 4 || WAVES == 8, "waves");
    static_assert(KT >= 1 && MT >= 1, "shape");
};

// acc[a] += T_tile(a, b) * B_tile(b) for the wave's K-tiles b; fragment di
// serves the pairs with a - 4 b = di - 4 (KT - 1) and is the four dwords at
// pr[4 di .. 4 di + 3] of the lane's shifted copy.
template <int N, int WAVES>
__device__ __forceinline__ void lat_mfma_block(const uint32_t *__restrict__ pr, v4i (&acc)[LatShape<N, WAVES>::MT],
                                               const v4i (&bf)[LatShape<N, WAVES>::KT])
{
    using S = LatShape<N, WAVES>;
    // Software pipeline: fragment di + 2 is requested before the MFMAs of
    // fragment di are issued (with one wave per SIMD, one fragment of MFMAs
    // does not cover a read's latency); sched_barrier keeps that order.
    auto frag = [&](int di) { return v4i{(int)pr[4 * di], (int)pr[4 * di + 1], (int)pr[4 * di + 2], (int)pr[4 * di + 3]}; };
    v4i fr = frag(0);
    v4i f1 = S::NDELTA > 1 ? frag(1) : fr;
    static_for<0, S::NDELTA>([&](auto dI) {
        constexpr int di = decltype(dI)::value;
        v4i f2 = f1;
        if constexpr (di + 2 < S::NDELTA) f2 = frag(di + 2);
        static_for<0, S::KT>([&](auto bI) {
            constexpr int b = decltype(bI)::value;
            constexpr int a = di - 4 * (S::KT - 1) + 4 * b;
            if constexpr (a >= 0 && a < S::MT) acc[a] = __builtin_amdgcn_mfma_i32_16x16x64_i8(fr, bf[b], acc[a], 0, 0, 0);
        });
        fr = f1;
        f1 = f2;
        __builtin_amdgcn_sched_barrier(0);
    });
}

template <int N, int WAVES>
__global__ __launch_bounds__(64 * WAVES, 1) void br_int8_lat_kernel(const uint8_t *__restrict__ bk8,
                                                                    const uint16_t *__restrict__ bars, int32_t n,
                                                                    uint32_t *__restrict__ ext)
{
    using S = LatShape<N, WAVES>;
    __shared__ __attribute__((aligned(16))) uint32_t acc_s[2][N];
    __shared__ __attribute__((aligned(16))) uint32_t xs[4 * S::XCOPY];   // copy r, row p, dword w

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int ks = wave % S::KS, pr = (wave / S::KS) & 1, c = wave / (2 * S::KS);
    const int col = lane & 15, g4 = lane >> 4;
    const int64_t g = blockIdx.x;   // the grid has exactly one workgroup per gate
    const uint16_t *bar = bars + g * (int64_t)(n + 1);

    // ACC = (0, X^{-bbar} v), v = (1/8) sum_j X^j.
    const uint32_t bb = bar[n];
    for (int m = tid; m < N; m += S::THREADS) {
        const uint32_t tt = ((uint32_t)m + bb) & (uint32_t)(2 * N - 1);
        acc_s[0][m] = 0u;
        acc_s[1][m] = tt < (uint32_t)N ? 0x20000000u : 0xE0000000u;
    }

    // A fragment source of this lane: byte offset s0 in X_p, block Q starting
    // N/2 bytes after block P (s0 >= 1, and the last fragment of Q ends at byte
    // 2N - 1), read as dword s0 / 4 of copy s0 & 3.
    const int s0 = N + (N / 2) * pr - 64 * S::KT * ks + col - 16 * g4 - 15 - 64 * (S::KT - 1);
    const uint32_t *xsrc = xs + (s0 & 3) * S::XCOPY + (s0 >> 2);

    // B fragments: limb kappa of half h of BK_i[p][q] (column 8 h + 4 q +
    // kappa) for k in the lane's 16-byte group, read reversed from the key
    // (byte N - 16 - k0 - 16 g4 .. + 15 for half 0, N/2 bytes lower for half 1).
    const int bhalf = col >> 3;
    const size_t bplane = (size_t)(col & 7) * (2 * N);   // plane (q, kappa) = ((col & 7) >> 2, col & 3)
    auto load_b = [&](int step, int row, v4i (&dst)[S::KT]) {
        const uint8_t *src = bk8 + ((size_t)step * BR_ROWS + row) * (2 * 4 * 2 * N) + bplane;
        static_for<0, S::KT>([&](auto bI) {
            constexpr int b = decltype(bI)::value;
            const int u0 = N - 16 - 64 * (S::KT * ks + b) - 16 * g4 - (N / 2) * bhalf;
            const u4 v = *reinterpret_cast<const u4 *>(src + u0);
            dst[b] = v4i{(int)v.x, (int)v.y, (int)v.z, (int)v.w};
        });
    };
    v4i nb[S::KT];
    load_b(0, 3 * c, nb);

    for (int i = 0; i < n; ++i) {
        const uint32_t a = bar[i];
        __syncthreads();   // ACC of the previous step complete; X consumed
        // Extended digit rows of D = X^a ACC_c - ACC_c. Item (c, k4) owns
        // coefficients 4 k4 .. 4 k4 + 3, i.e. dword k4 (negated digits) and
        // dword N/4 + k4 (digits) of X_p; it also takes the digits of the next
        // group, which the shifted copies of those dwords reach into.
        for (int e = tid; e < N / 2; e += S::THREADS) {
            const int cc = e / (N / 4), k4 = e - cc * (N / 4);
            const bool last = k4 + 1 == N / 4;
            uint32_t word[2][3];   // digit fields + 64 of groups k4 and k4 + 1 (mod N/4), one byte each
            static_for<0, 2>([&](auto hI) {
                constexpr int h = decltype(hI)::value;
                const int kg = h == 0 ? k4 : (last ? 0 : k4 + 1);
                const u4 own = *reinterpret_cast<const u4 *>(&acc_s[cc][4 * kg]);
                const uint32_t un[4] = {own.x, own.y, own.z, own.w};
                word[h][0] = word[h][1] = word[h][2] = 0u;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const uint32_t tt = ((uint32_t)(4 * kg + t) - a) & (uint32_t)(2 * N - 1);
                    uint32_t v = acc_s[cc][tt & (uint32_t)(N - 1)];
                    v = (tt & (uint32_t)N) ? 0u - v : v;
                    const uint32_t y = v - un[t] + kDigitOffset;
#pragma unroll
                    for (int j = 0; j < 3; ++j) word[h][j] |= ((y >> (32 - 7 * (j + 1))) & 127u) << (8 * t);
                }
            });
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                // bytes f = d + 64 in [0, 128): d = (f + 64) ^ 0x80, -d = (0xC0 - f) ^ 0x80, no carries
                const uint32_t pos_lo = (word[0][j] + 0x40404040u) ^ 0x80808080u;
                const uint32_t neg_lo = (0xC0C0C0C0u - word[0][j]) ^ 0x80808080u;
                const uint32_t pos_hi = (word[1][j] + 0x40404040u) ^ 0x80808080u;
                const uint32_t neg_hi = (0xC0C0C0C0u - word[1][j]) ^ 0x80808080u;
                // the dword after the negated half's last one is the first of the
                // digit half; nothing is read past the digit half's last byte
                const uint32_t next_neg = last ? pos_hi : neg_hi;
                const uint32_t next_pos = last ? 0u : pos_hi;
                uint32_t *row = xs + (3 * cc + j) * S::XD;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    row[r * S::XCOPY + k4] = r == 0 ? neg_lo : __builtin_amdgcn_alignbyte(next_neg, neg_lo, (uint32_t)r);
                    row[r * S::XCOPY + N / 4 + k4] = r == 0 ? pos_lo : __builtin_amdgcn_alignbyte(next_pos, pos_lo, (uint32_t)r);
                }
            }
        }
        __syncthreads();   // digit rows visible, every read of ACC done

        v4i acc[S::MT];
        static_for<0, S::MT>([&](auto tI) { acc[decltype(tI)::value] = v4i{0, 0, 0, 0}; });
        // With 8 waves, waves w and w + 4 share a SIMD and do the same work;
        // the arbiter issues the older one first, so the younger raises its
        // priority for the first two of its three digit rows and the pair
        // reaches the atomic adds together (9.29 against 9.48 ms for 64 gates;
        // raised for one row 9.34, for all three 9.41).
        if (WAVES == 8 && wave >= 4) __builtin_amdgcn_s_setprio(1);
#pragma unroll 1
        for (int j = 0; j < 3; ++j) {
            if (j == 2) __builtin_amdgcn_s_setprio(0);
            v4i bf[S::KT];
            static_for<0, S::KT>([&](auto bI) { bf[decltype(bI)::value] = nb[decltype(bI)::value]; });
            // next (step, row); past the last step reload step 0 (unused)
            const int ni = j < 2 ? i : (i + 1 < n ? i + 1 : 0);
            load_b(ni, 3 * c + (j < 2 ? j + 1 : 0), nb);
            lat_mfma_block<N, WAVES>(xsrc + (3 * c + j) * S::XD, acc, bf);
        }
        // The block product's column 8 h + 4 q + kappa holds limb kappa of
        // (block x key half h) for output q: sum_kappa 2^(8 kappa) C[m][.].
        // The four limbs of an output row sit in the four lanes of a quad,
        // each lane holding rows 4 g4 + e, e = 0..3. A reduce-scatter over the
        // quad (exchange with lane ^ 1, then lane ^ 2) leaves lane kappa with
        // the full sum of row e = kappa. Block P times half h goes to output
        // half h (+P k0 into y0, +P k1 into y1); block Q times half 0 goes to
        // y1 (+Q k0) and times half 1 to y0 (-Q k1).
        const uint32_t lsh = 8u * (uint32_t)(lane & 3);
        const bool odd = (lane & 1) != 0, hi2 = (lane & 2) != 0;
        const int out_half = pr ? 1 - bhalf : bhalf;
        const bool negate = pr && bhalf;
        uint32_t *accq = acc_s[(lane >> 2) & 1] + (N / 2) * out_half + 4 * g4 + (lane & 3);
        static_for<0, S::MT>([&](auto tI) {
            constexpr int t = decltype(tI)::value;
            const uint32_t v0 = (uint32_t)acc[t][0] << lsh, v1 = (uint32_t)acc[t][1] << lsh;
            const uint32_t v2 = (uint32_t)acc[t][2] << lsh, v3 = (uint32_t)acc[t][3] << lsh;
            // The selects come before the cross-lane moves, which every lane
            // executes: a DPP read of a lane outside the exec mask yields 0,
            // so the moves must not sit under lane-dependent branches.
            // keep rows e = 2h + (lane & 1), pass the other two to lane ^ 1 (quad_perm [1,0,3,2])
            const uint32_t z0 = (odd ? v1 : v0) + (uint32_t)__builtin_amdgcn_mov_dpp((int)(odd ? v0 : v1), 0xB1, 0xF, 0xF, false);
            const uint32_t z1 = (odd ? v3 : v2) + (uint32_t)__builtin_amdgcn_mov_dpp((int)(odd ? v2 : v3), 0xB1, 0xF, 0xF, false);
            // keep row e = lane & 3, pass the other to lane ^ 2 (quad_perm [2,3,0,1])
            const uint32_t r = (hi2 ? z1 : z0) + (uint32_t)__builtin_amdgcn_mov_dpp((int)(hi2 ? z0 : z1), 0x4E, 0xF, 0xF, false);
            atomicAdd(accq + 16 * t, negate ? 0u - r : r);
        });
    }
    __syncthreads();

    // Sample extraction: a'_0 = A_0, a'_j = -A_{N-j}, b' = B_0.
    uint32_t *out = ext + g * (N + 1);
    for (int jj = tid; jj <= N; jj += S::THREADS) {
        uint32_t v;
        if (jj == 0) v = acc_s[0][0];
        else if (jj == N) v = acc_s[1][0];
        else v = 0u - acc_s[0][N - jj];
        out[jj] = v;
    }
}

template <int N, int WAVES>
int launch_shape(const cemu_cloud_key *ck, const uint16_t *bars, int64_t B, uint32_t *ext, hipStream_t s)
{
    const int n = ck->p.n;
    auto one_gate = [&](const uint16_t *b, int64_t cnt, uint32_t *x) {
        hipLaunchKernelGGL((br_int8_lat_kernel<N, WAVES>), dim3((unsigned)cnt), dim3(64 * WAVES), 0, s, ck->d_bk8, b, n,
                           x);
    };
    if (ck->tuning.int8_gates_per_wg == 1) {
        one_gate(bars, B, ext);
        return CEMU_OK;
    }
    // The 16-gate kernel runs one workgroup per CU, so a launch proceeds in
    // rounds of 16 * CUs gates and a round costs the same however few of its
    // workgroups are busy (75-87 ms on MI355X). A short tail behind full
    // rounds goes to the one-gate kernel instead (6.2-7.1 ms per CUs gates):
    // up to 12 * CUs gates. Outputs do not depend on the shape.
    const int64_t cus = ck->num_cus;
    int64_t full = B;
    if (cus > 0) {
        const int64_t round = BR_G * cus;
        const int64_t r = B % round;
        if (B >= round && r > 0 && r <= 12 * cus) full = B - r;
    }
    const int64_t blocks = (full + BR_G - 1) / BR_G;
    if constexpr (WAVES == 8)
        hipLaunchKernelGGL((br_int8_res_kernel<N>), dim3((unsigned)blocks), dim3(512), 0, s, ck->d_bk8, bars, n, full, ext);
    else
        hipLaunchKernelGGL((br_int8_kernel<N, WAVES>), dim3((unsigned)blocks), dim3(64 * WAVES), 0, s, ck->d_bk8, bars,
                           n, full, ext);
    if (full < B) one_gate(bars + full * (int64_t)(n + 1), B - full, ext + full * (int64_t)(N + 1));
    return CEMU_OK;
}

}  // namespace

int br_int8_batch_ok(const cemu_cloud_key *ck, int64_t B)
{
    // one workgroup per gate (latency kernel) or per BR_G gates
    const int64_t blocks = ck->tuning.int8_gates_per_wg == 1 ? B : (B + BR_G - 1) / BR_G;
    if (B < 0 || blocks * 64 * ck->tuning.int8_waves > (int64_t)0xffffffff)
        return fail(CEMU_ERR_RANGE, "batch too large for one launch");
    return CEMU_OK;
}

int launch_br_int8(const cemu_cloud_key *ck, const uint16_t *bars, int64_t B, uint32_t *ext, hipStream_t s)
{
    if (const int rc = br_int8_batch_ok(ck, B)) return rc;
    if (B == 0) return CEMU_OK;
    const int waves = ck->tuning.int8_waves;   // 4 or 8 (validated by cemu_set_tuning)
    int rc;
    if (ck->p.N == 1024) rc = waves == 8 ? launch_shape<1024, 8>(ck, bars, B, ext, s) : launch_shape<1024, 4>(ck, bars, B, ext, s);
    else if (ck->p.N == 512) rc = waves == 8 ? launch_shape<512, 8>(ck, bars, B, ext, s) : launch_shape<512, 4>(ck, bars, B, ext, s);
    else return fail(CEMU_ERR_UNSUPPORTED, "N must be 512 or 1024");
    if (rc) return rc;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(CEMU_ERR_HIP, std::string("br_int8_kernel launch: ") + hipGetErrorString(e));
    return CEMU_OK;
}

}  // namespace cemu
