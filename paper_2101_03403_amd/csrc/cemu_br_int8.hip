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
// consecutive bytes of R, fetched as 5 aligned dwords from LDS and shifted
// with v_alignbyte. A 16x64 tile of T depends only on (k0 - m0), so each
// generated fragment is reused for every (M-tile, K-tile) pair on that
// diagonal: MT*KT / NDELTA = 512/92 (N = 1024) MFMAs per generated fragment.
//
// Waves: 4 per workgroup; wave w computes output component q = w/2 for rows
// [h*N/2, (h+1)*N/2), h = w%2, and keeps the step's running sum in registers.
#include <hip/hip_runtime.h>

#include "cemu_kernels.h"

namespace cemu {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int BR_G = 16;         // gates per workgroup = MFMA N dimension
constexpr int BR_THREADS = 256;  // 4 waves
constexpr int BR_ROWS = 6;       // (k+1) * l digit rows, k = 1, l = 3
constexpr int LDS_PAD = 4;       // words of padding per accumulator row

template <int N>
struct BrShape {
    static constexpr int HALF = N / 2;                          // rows per wave
    static constexpr int MT = HALF / 16;                        // 16-row M-tiles per wave
    static constexpr int KT = N / 64;                           // 64-wide K-tiles per digit row
    static constexpr int ROW = N + LDS_PAD;                     // LDS words per (component, gate)
    static constexpr int RB = 2 * N;                            // bytes of one limb sequence R
    static constexpr int STAGE_BYTES = 2 * 4 * RB;              // R for one digit row: (q, limb)
    static constexpr int NDELTA = (MT - 1) + 4 * (KT - 1) + 1;  // distinct fragments per block
    static constexpr int PRE = STAGE_BYTES / (BR_THREADS * 16); // uint4 per thread per stage
};

// OFF = sum_{j=1..3} (Bg/2) 2^(32-7j) + 2^(32-21-1): adding it turns the
// signed rounded digits into plain bit fields: d_j = ((x+OFF) >> (32-7j)) & 127) - 64.
constexpr uint32_t kDigitOffset = 0x81020400u;

// Digits of level j for the 16 gates, in MFMA B-operand layout: lane
// (gate = lane&15, kgroup = lane>>4), K-tile b, byte e holds digit of
// coefficient k = 64b + 16*kgroup + e of  X^a * P - P,  P = this lane's
// accumulator component.
template <int N>
__device__ __forceinline__ void compute_bfrag(const uint32_t *__restrict__ row, uint32_t a, uint32_t sh, int g4,
                                              v4i (&bf)[BrShape<N>::KT])
{
#pragma unroll
    for (int b = 0; b < BrShape<N>::KT; ++b) {
        const int k0 = 64 * b + 16 * g4;
        const uint4 *up = reinterpret_cast<const uint4 *>(row + k0);
        uint4 u4[4];
#pragma unroll
        for (int d = 0; d < 4; ++d) u4[d] = up[d];
        uint32_t packed[4];
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            const uint32_t un[4] = {u4[d].x, u4[d].y, u4[d].z, u4[d].w};
            uint32_t word = 0;
#pragma unroll
            for (int e4 = 0; e4 < 4; ++e4) {
                const uint32_t k = (uint32_t)(k0 + 4 * d + e4);
                const uint32_t tt = (k - a) & (uint32_t)(2 * N - 1);
                uint32_t v = row[tt & (uint32_t)(N - 1)];
                v = (tt & (uint32_t)N) ? 0u - v : v;
                const uint32_t y = v - un[e4] + kDigitOffset;
                word |= ((y >> sh) & 127u) << (8 * e4);
            }
            // bytes x in [0,128) hold digit + 64; (x + 64) ^ 0x80 = x - 64 mod 256, no carries
            packed[d] = (word + 0x40404040u) ^ 0x80808080u;
        }
        bf[b] = v4i{(int)packed[0], (int)packed[1], (int)packed[2], (int)packed[3]};
    }
}

// acc[a] += T_tile(a, b) * D_tile(b) for all (a, b), one limb, fragments
// generated once per diagonal delta = 4b - a.
template <int N>
__device__ __forceinline__ void mfma_block(const uint32_t *__restrict__ pr, uint32_t shift,
                                           v4i (&acc)[BrShape<N>::MT], const v4i (&bf)[BrShape<N>::KT])
{
    using S = BrShape<N>;
    uint32_t w0 = pr[0];
#pragma unroll
    for (int di = 0; di < S::NDELTA; ++di) {
        const uint32_t w1 = pr[4 * di + 1], w2 = pr[4 * di + 2], w3 = pr[4 * di + 3], w4 = pr[4 * di + 4];
        const v4i fr = v4i{(int)__builtin_amdgcn_alignbyte(w1, w0, shift), (int)__builtin_amdgcn_alignbyte(w2, w1, shift),
                           (int)__builtin_amdgcn_alignbyte(w3, w2, shift), (int)__builtin_amdgcn_alignbyte(w4, w3, shift)};
#pragma unroll
        for (int b = 0; b < S::KT; ++b) {
            const int a = 4 * b - (di - (S::MT - 1));
            if (a >= 0 && a < S::MT) acc[a] = __builtin_amdgcn_mfma_i32_16x16x64_i8(fr, bf[b], acc[a], 0, 0, 0);
        }
        w0 = w4;
    }
}

template <int N>
__global__ __launch_bounds__(BR_THREADS, 1) void br_int8_kernel(const uint8_t *__restrict__ bk8,
                                                                const uint16_t *__restrict__ bars, int32_t n,
                                                                int64_t B, uint32_t *__restrict__ ext)
{
    using S = BrShape<N>;
    __shared__ __attribute__((aligned(16))) uint32_t acc_s[2][BR_G][S::ROW];
    __shared__ __attribute__((aligned(16))) uint32_t rst[S::STAGE_BYTES / 4];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int q = wave >> 1, h = wave & 1;
    const int gl = lane & 15, g4 = lane >> 4;
    const int64_t g0 = (int64_t)blockIdx.x * BR_G;
    const int64_t barrow = (int64_t)n + 1;
    const bool live = g0 + gl < B;
    const uint16_t *mybars = bars + (g0 + gl) * barrow;

    // ACC = (0, X^{-bbar} v), v = (1/8) sum_j X^j.
    for (int e = tid; e < BR_G * N; e += BR_THREADS) {
        const int g = e / N, m = e - (e / N) * N;
        const uint32_t bb = (g0 + g < B) ? (uint32_t)bars[(g0 + g) * barrow + n] : 0u;
        const uint32_t tt = ((uint32_t)m + bb) & (uint32_t)(2 * N - 1);
        acc_s[0][g][m] = 0u;
        acc_s[1][g][m] = tt < (uint32_t)N ? 0x20000000u : 0xE0000000u;
    }

    // Lane's A-fragment source: s0 = N-1 - h*N/2 - r + 16*kgroup - 16*(MT-1) >= 0.
    const int s0 = (N - 1) - h * S::HALF - gl + 16 * g4 - 16 * (S::MT - 1);
    const uint32_t frag_shift = (uint32_t)(s0 & 3);
    const int frag_dw = s0 >> 2;

    uint4 pre[S::PRE];
    auto load_stage = [&](int i, int p) {
        const uint4 *src = reinterpret_cast<const uint4 *>(bk8 + ((size_t)i * BR_ROWS + p) * S::STAGE_BYTES);
#pragma unroll
        for (int k = 0; k < S::PRE; ++k) pre[k] = src[tid + k * BR_THREADS];
    };
    load_stage(0, 0);

    uint32_t a_cur = live ? (uint32_t)mybars[0] : 0u;
    v4i total[S::MT];

    for (int i = 0; i < n; ++i) {
        const uint32_t a_next = (live && i + 1 < n) ? (uint32_t)mybars[i + 1] : 0u;
#pragma unroll
        for (int t = 0; t < S::MT; ++t) total[t] = v4i{0, 0, 0, 0};

#pragma unroll 1
        for (int p = 0; p < BR_ROWS; ++p) {
            __syncthreads();  // previous users of rst are done; ACC updates visible
            {
                uint4 *dst = reinterpret_cast<uint4 *>(rst);
#pragma unroll
                for (int k = 0; k < S::PRE; ++k) dst[tid + k * BR_THREADS] = pre[k];
            }
            {
                int ni = i, np = p + 1;
                if (np == BR_ROWS) {
                    np = 0;
                    ++ni;
                }
                if (ni < n) load_stage(ni, np);
            }
            __syncthreads();  // stage visible

            const int c = p / 3, j = p - (p / 3) * 3;
            v4i bf[S::KT];
            compute_bfrag<N>(&acc_s[c][gl][0], a_cur, (uint32_t)(32 - 7 * (j + 1)), g4, bf);

            v4i acc[S::MT];
#pragma unroll
            for (int t = 0; t < S::MT; ++t) acc[t] = v4i{0, 0, 0, 0};
#pragma unroll 1
            for (int kappa = 3; kappa >= 0; --kappa) {
                if (kappa != 3) {
#pragma unroll
                    for (int t = 0; t < S::MT; ++t) acc[t] = acc[t] << 8;
                }
                const uint32_t *pr = rst + (q * 4 + kappa) * (S::RB / 4) + frag_dw;
                mfma_block<N>(pr, frag_shift, acc, bf);
            }
#pragma unroll
            for (int t = 0; t < S::MT; ++t) total[t] += acc[t];
        }
        __syncthreads();  // every wave has finished reading ACC for this step
#pragma unroll
        for (int t = 0; t < S::MT; ++t) {
            uint4 *ptr = reinterpret_cast<uint4 *>(&acc_s[q][gl][h * S::HALF + 16 * t + 4 * g4]);
            uint4 v = *ptr;
            v.x += (uint32_t)total[t][0];
            v.y += (uint32_t)total[t][1];
            v.z += (uint32_t)total[t][2];
            v.w += (uint32_t)total[t][3];
            *ptr = v;
        }
        a_cur = a_next;
    }
    __syncthreads();

    // Sample extraction: a'_0 = A_0, a'_j = -A_{N-j}, b' = B_0.
    for (int e = tid; e < BR_G * (N + 1); e += BR_THREADS) {
        const int g = e / (N + 1), jj = e - (e / (N + 1)) * (N + 1);
        if (g0 + g >= B) continue;
        uint32_t v;
        if (jj == 0) v = acc_s[0][g][0];
        else if (jj == N) v = acc_s[1][g][0];
        else v = 0u - acc_s[0][g][N - jj];
        ext[(g0 + g) * (N + 1) + jj] = v;
    }
}

}  // namespace

int launch_br_int8(const cemu_cloud_key *ck, const uint16_t *bars, int64_t B, uint32_t *ext, hipStream_t s)
{
    const int64_t blocks = (B + BR_G - 1) / BR_G;
    if (blocks > 0x7fffffff) return fail(CEMU_ERR_RANGE, "batch too large");
    if (ck->p.N == 1024)
        hipLaunchKernelGGL(br_int8_kernel<1024>, dim3((unsigned)blocks), dim3(BR_THREADS), 0, s, ck->d_bk8, bars,
                           ck->p.n, B, ext);
    else if (ck->p.N == 512)
        hipLaunchKernelGGL(br_int8_kernel<512>, dim3((unsigned)blocks), dim3(BR_THREADS), 0, s, ck->d_bk8, bars,
                           ck->p.n, B, ext);
    else
        return fail(CEMU_ERR_UNSUPPORTED, "N must be 512 or 1024");
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(CEMU_ERR_HIP, std::string("br_int8_kernel launch: ") + hipGetErrorString(e));
    return CEMU_OK;
}

int launch_br_fft(cemu_cloud_key *, const uint16_t *, int64_t, uint32_t *, hipStream_t)
{
    return fail(CEMU_ERR_UNSUPPORTED, "the FFT64 form is not built yet");
}

}  // namespace cemu
