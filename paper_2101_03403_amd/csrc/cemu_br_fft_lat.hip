// Latency kernel (narrow batches): one gate per workgroup of 8 waves. Six
// waves, one per gadget digit, run the 6 forward transforms of a step side
// by side and leave their spectra in LDS; every wave then forms, for one
// frequency slot, both outputs' sums over the six rows (in a fixed row
// order, its key values prefetched into registers a step ahead), and two
// waves run the two inverse transforms. A step then costs about three
// transform latencies instead of eight.
//
// This file is compiled with the machine scheduler that forms the longest
// clauses of memory instructions (-amdgpu-sched-strategy=max-memory-clause,
// set in the build): for this kernel it shortens a step by about 2.6 %
// (measured); the other kernels are faster with the default scheduler.
#include <hip/hip_runtime.h>

#include "cemu_fft.h"
#include "cemu_kernels.h"

namespace cemu {
namespace {

// ACC component c is kept as one 16-byte record per coefficient pair
// (j, j + N/2), j < N/2: (R_j, R_{j+N/2}, ACC_j, ACC_{j+N/2}) with
// R = X^a ACC for the rotation a of the step about to run, so a digit wave
// gets D = R - ACC at its 16 coefficients from 8 aligned 16-byte reads.
// The rotation amounts are known in advance (the bars), so the waves that
// update ACC write R for the next step directly: ACC_j and ACC_{j+N/2} land
// at k = (j + a) mod 2N and k + N/2, i.e. in one record r = k mod N/2, as
// (f, s) = (v0, v1), (-v1, v0), (-v0, -v1) or (v1, -v0) for k / (N/2) =
// 0, 1, 2, 3 (negacyclic wrap).
//
// A step: waves 0..5 (digit row p = wave) decompose and transform their
// digit row and write its spectrum to their region; then every wave w takes
// frequency slot w of all six spectra and forms both outputs' sums
// sum_p X_p K_{p,q} there (its twelve key values prefetched a step ahead);
// then waves 6 and 7 run the inverse transforms of outputs 0 and 1. Only
// the spectra (8 KiB per row) and the sums cross LDS, not per-row products.
__global__ __launch_bounds__(64 * LAT_WAVES, 1) void br_fft_lat_kernel(const d2 *__restrict__ spec,
                                                                      const uint16_t *__restrict__ bars, int32_t n,
                                                                      uint32_t *__restrict__ ext)
{
    static_assert(FH <= SCR, "a spectrum fits a region");
    __shared__ __attribute__((aligned(16))) uint32_t zacc[2][4 * FH];
    // region of wave w: its transpose scratch during a transform, then (digit
    // waves) its spectrum in (slot, lane) order
    __shared__ d2 region[LAT_WAVES][SCR];
    __shared__ d2 sums[2][FH];                 // output q's spectrum, (slot, lane) order
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = tid >> 6;
    const bool digit_wave = w < 6;
    const int p = digit_wave ? w : 0;          // digit row of a digit wave: component c, digit jj
    const int c = p / 3, jj = p - 3 * c;
    const uint32_t sh = (uint32_t)(32 - 7 * (jj + 1));
    const int q_inv = w - 6;                   // output of an inverse wave (waves 6, 7)
    const int64_t g = blockIdx.x;              // the grid has exactly one workgroup per gate
    d2 *scr = region[w];
    const uint16_t *bar = bars + g * (int64_t)(n + 1);
    const Tw t0 = make_tw(lane);
    Tw t = t0;

    // ACC = (0, X^{-bbar} v) with the records of step 0 (R = X^{a_0} ACC)
    const uint32_t bb = bar[n], a0 = bar[0];
    auto tv = [&](uint32_t m) {   // coefficient m < N of X^{-bbar} v
        return ((m + bb) & (uint32_t)(2 * FN - 1)) < (uint32_t)FN ? 0x20000000u : 0xE0000000u;
    };
    for (int e = tid; e < FH; e += 64 * LAT_WAVES) {
        uint32_t r[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const uint32_t tt = ((uint32_t)(e + h * FH) - a0) & (uint32_t)(2 * FN - 1);
            const uint32_t v = tv(tt & (uint32_t)(FN - 1));
            r[h] = (tt & (uint32_t)FN) ? 0u - v : v;
        }
        *reinterpret_cast<uint4 *>(&zacc[0][4 * e]) = uint4{0u, 0u, 0u, 0u};
        *reinterpret_cast<uint4 *>(&zacc[1][4 * e]) = uint4{r[0], r[1], tv((uint32_t)e), tv((uint32_t)(e + FH))};
    }
    // the two inverse waves keep their component's own 16 coefficients
    // (j = lane + 64 m + 512 h) in registers
    uint32_t mine[16];
    static_for<0, 16>([&](auto sI) {
        constexpr int sl = decltype(sI)::value;
        const uint32_t tt = ((uint32_t)(lane + 64 * sl) + bb) & (uint32_t)(2 * FN - 1);
        mine[sl] = q_inv == 1 ? (tt < (uint32_t)FN ? 0x20000000u : 0xE0000000u) : 0u;
    });
    // key values of this wave's slot for step 0: kr[2 p + q] = K_{p,q}[slot w, lane]
    d2 kr[12];
    {
        const d2 *src = spec + w * 64 + lane;
        static_for<0, 12>([&](auto kI) { kr[decltype(kI)::value] = src[decltype(kI)::value * FH]; });
    }
    __syncthreads();

    const uint4 *zc = reinterpret_cast<const uint4 *>(zacc[c]) + lane;
    for (int i = 0; i < n; ++i) {
        // the next step's rotation, applied when the ACC records are written back
        const uint32_t a_next = i + 1 < n ? (uint32_t)bar[i + 1] : 0u;
        launder(t.tw); launder(t.f1); launder(t.f2); launder(t.i2c); launder(t.i2b);
        if (digit_wave) {
            // waves 4 and 5 share a SIMD with waves 0 and 1, which the arbiter
            // issues first; raising them until the first transpose of their
            // forward transform lets each pair finish that phase together
            if (p >= 4) __builtin_amdgcn_s_setprio(1);
            // digit jj of D = X^a ACC_c - ACC_c at this lane's 16 coefficients
            d2 x[8];
            // all eight records requested before the first is used (left to
            // itself the compiler keeps two reads in flight, exposing their latency)
            uint4 zw[8];
            static_for<0, 8>([&](auto mI) { zw[decltype(mI)::value] = zc[64 * decltype(mI)::value]; });
            __builtin_amdgcn_sched_barrier(0);
            static_for<0, 8>([&](auto mI) {
                constexpr int m = decltype(mI)::value;
                const uint4 zv = zw[m];
                const uint32_t d0 = zv.x - zv.z + kDigitOffset;
                const uint32_t d1 = zv.y - zv.w + kDigitOffset;
                const double lo = (double)((int32_t)((d0 >> sh) & 127u) - 64);
                const double hi = (double)((int32_t)((d1 >> sh) & 127u) - 64);
                x[m] = cmul(d2{lo, hi}, twist_slot(m));
            });
            __builtin_amdgcn_sched_barrier(0);
            fft_fwd<true>(x, scr, lane, t);
            __builtin_amdgcn_sched_barrier(0);
            // the spectrum, into this wave's region (its transform is done;
            // LDS ops of a wave are ordered)
            wave_lds_fence();
            static_for<0, 8>([&](auto sI) { scr[decltype(sI)::value * 64 + lane] = x[decltype(sI)::value]; });
        }
        __syncthreads();   // spectra visible
        {
            // slot w of both outputs: the six rows in row order
            d2 sa = d2{0.0, 0.0}, sb = d2{0.0, 0.0};
            static_for<0, 6>([&](auto rI) {
                constexpr int r = decltype(rI)::value;
                const d2 xr = region[r][w * 64 + lane];
                sa = cmac(sa, xr, kr[2 * r]);
                sb = cmac(sb, xr, kr[2 * r + 1]);
            });
            sums[0][w * 64 + lane] = sa;
            sums[1][w * 64 + lane] = sb;
            // the next step's key values (past the last step: step 0, unused)
            const int ni = i + 1 < n ? i + 1 : 0;
            const d2 *src = spec + (int64_t)ni * 6 * STAGE_D2 + w * 64 + lane;
            static_for<0, 12>([&](auto kI) { kr[decltype(kI)::value] = src[decltype(kI)::value * FH]; });
        }
        __syncthreads();   // sums visible
        if (!digit_wave) {
            // output q: inverse transform, untwist, round and accumulate into
            // ACC_q (scratch: this wave's own region)
            d2 y[8];
            static_for<0, 8>([&](auto sI) { y[decltype(sI)::value] = sums[q_inv][decltype(sI)::value * 64 + lane]; });
            fft_inv(y, scr, lane, t);
            uint32_t *zq = zacc[q_inv];
            static_for<0, 8>([&](auto mI) {
                constexpr int m = decltype(mI)::value;
                const d2 z = cmul(y[m], cconj(twist_slot(m)));
                const uint32_t v0 = mine[m] + round_mod32(z.x);
                const uint32_t v1 = mine[m + 8] + round_mod32(z.y);
                mine[m] = v0;
                mine[m + 8] = v1;
                const uint32_t j = (uint32_t)(lane + 64 * m);
                *reinterpret_cast<uint2 *>(&zq[4 * j + 2]) = uint2{v0, v1};
                // this pair rotated by the next step's amount (unused after the last step)
                const uint32_t k = (j + a_next) & (uint32_t)(2 * FN - 1);
                const uint32_t quad = k / FH;
                const uint32_t f = (quad & 1u) ? v1 : v0, sc = (quad & 1u) ? v0 : v1;
                const uint32_t fr = (quad == 1u || quad == 2u) ? 0u - f : f;
                const uint32_t sr = (quad >= 2u) ? 0u - sc : sc;
                *reinterpret_cast<uint2 *>(&zq[4 * (k & (uint32_t)(FH - 1))]) = uint2{fr, sr};
            });
        }
        __syncthreads();   // ACC updated
    }

    // sample extraction
    uint32_t *e = ext + g * (FN + 1);
    for (int j = tid; j <= FN; j += 64 * LAT_WAVES) {
        uint32_t v;
        auto accw = [&](int q, int k) { return zacc[q][4 * (k & (FH - 1)) + 2 + (k >= FH)]; };
        if (j == 0) v = accw(0, 0);
        else if (j == FN) v = accw(1, 0);
        else v = 0u - accw(0, FN - j);
        e[j] = v;
    }
}

}  // namespace

void launch_br_fft_lat(const double *spec, const uint16_t *bars, int32_t n, int64_t cnt, uint32_t *ext,
                       hipStream_t s)
{
    hipLaunchKernelGGL(br_fft_lat_kernel, dim3((unsigned)cnt), dim3(64 * LAT_WAVES), 0, s,
                       reinterpret_cast<const d2 *>(spec), bars, n, ext);
}

}  // namespace cemu
