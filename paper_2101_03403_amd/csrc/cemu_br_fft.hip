// Blind rotation with FP64 negacyclic-FFT products (gfx950): key-spectrum
// preparation, the throughput kernel and the launcher of both FFT shapes. The
// transform itself is in cemu_fft.h; the latency kernel, built with its own
// scheduling options, in cemu_br_fft_lat.hip.
//
// Throughput kernel: one wave per gate, FG = 8 (default) or 4 gates per
// workgroup: each wave keeps its accumulator (2 x N u32, as 8-byte records of
// the coefficient pair (j, j + N/2)) and its FFT transpose scratch in LDS; the
// key spectra of one digit row (16 KiB) are staged in LDS once per workgroup,
// prefetched through registers one row ahead.
#include <hip/hip_runtime.h>

#include "cemu_fft.h"
#include "cemu_kernels.h"

namespace cemu {
namespace {

// Key spectrum preparation: one wave per (step i, digit row r, component q).
// Reads the int8-limb key (R[u] = limb(E[2N-1-u]), BK[m] at u = N-1-m),
// centres each Torus32 coefficient, folds, twists and transforms.
__global__ __launch_bounds__(64) void bk_fft_prepare_kernel(const uint8_t *__restrict__ bk8, d2 *__restrict__ spec)
{
    __shared__ d2 scr[SCR];
    const int lane = threadIdx.x;
    const int64_t poly = blockIdx.x;            // (i*6 + r)*2 + q
    const uint8_t *base = bk8 + poly * 4 * (2 * FN);
    const Tw t = make_tw(lane);
    d2 x[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        double v[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int j = lane + 64 * m + h * FH;
            const int u = FN - 1 - j;
            uint32_t val = 0;
#pragma unroll
            for (int k = 3; k >= 0; --k) val = (val << 8) + (uint32_t)(int32_t)(int8_t)base[k * (2 * FN) + u];
            v[h] = (double)(int32_t)val;
        }
        x[m] = cmul(d2{v[0], v[1]}, twist_slot(m));
    }
    fft_fwd(x, scr, lane, t);
    d2 *dst = spec + poly * FH;
#pragma unroll
    for (int s = 0; s < 8; ++s) dst[s * 64 + lane] = x[s];
}

// FG = gates (waves) per workgroup: 8 (two waves per SIMD, 256 registers
// each) or 4 (one wave per SIMD, 512 registers).
//
// Issue balance: waves w and w + FG/2 share a SIMD, and the hardware issues
// the older one (w) first, so left alone it runs ahead through every phase
// and the younger one ends each phase alone, at the issue rate of a single
// wave, while w waits at the next barrier. The younger wave raises its
// priority for the first half of each phase -- the digit extraction and the
// forward transform up to its first transpose, the first half of the
// products, the first of the two inverse transforms -- so that the pair
// reaches the end of the phase together.
//   4096 gates: 20.7 ms against 24.55 ms without it (a whole-phase boost,
//   other split points, or an extra barrier instead were slower).
template <int FG>
__global__ __launch_bounds__(64 * FG, 1) void br_fft_kernel(const d2 *__restrict__ spec,
                                                           const uint16_t *__restrict__ bars, int32_t n, int64_t B,
                                                           uint32_t *__restrict__ ext)
{
    constexpr int F_THREADS = 64 * FG;
    constexpr int F_PRE = STAGE_D2 / F_THREADS;   // d2 per thread per stage
    // ACC component c of a gate: record r < N/2 holds (ACC_r, ACC_{r+N/2}),
    // so a lane reads or updates its coefficient pair (j, j + N/2) with one
    // 8-byte access, and the rotated pair of a step is one record too
    __shared__ uint2 acc_all[FG][2][FH];
    __shared__ d2 scr_all[FG][SCR];
    __shared__ d2 kst[STAGE_D2];               // key spectra of the current digit row
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t g = (int64_t)blockIdx.x * FG + wave;
    const bool live = g < B;
    uint2(&acc)[2][FH] = acc_all[wave];
    d2 *scr = scr_all[wave];
    const uint16_t *bar = bars + (live ? g : 0) * (int64_t)(n + 1);
    const Tw t0 = make_tw(lane);
    Tw t = t0;

    // ACC = (0, X^{-bbar} v)
    const uint32_t bb = live ? bar[n] : 0u;
    auto tv = [&](uint32_t m) {   // coefficient m < N of X^{-bbar} v
        return ((m + bb) & (uint32_t)(2 * FN - 1)) < (uint32_t)FN ? 0x20000000u : 0xE0000000u;
    };
    for (int r = lane; r < FH; r += 64) {
        acc[0][r] = uint2{0u, 0u};
        acc[1][r] = uint2{tv((uint32_t)r), tv((uint32_t)(r + FH))};
    }

    d2 pre[F_PRE];
    static_for<0, F_PRE>([&](auto kI) { pre[decltype(kI)::value] = spec[tid + decltype(kI)::value * F_THREADS]; });

    uint32_t a_next = live ? bar[0] : 0u;
    for (int i = 0; i < n; ++i) {
        const uint32_t a = a_next;
        if (live && i + 1 < n) a_next = bar[i + 1];
        launder(t.tw); launder(t.f1); launder(t.f2); launder(t.i2c); launder(t.i2b);
        d2 outA[8], outB[8];
        static_for<0, 8>([&](auto sI) {
            outA[decltype(sI)::value] = d2{0.0, 0.0};
            outB[decltype(sI)::value] = d2{0.0, 0.0};
        });
#pragma unroll 1
        for (int c = 0; c < 2; ++c) {
            // D = X^a ACC_c - ACC_c at this lane's 16 coefficients (+ digit offset, field top bits flipped).
            // Coefficients j and j + N/2 of X^a ACC come from ACC at t = j - a and
            // t + N/2 (mod 2N), which share the record t mod N/2; the quadrant
            // t / (N/2) says which half each takes and which are negated
            // (X^N = -1): (v0, v1) = (x, y), (y, -x), (-x, -y), (-y, x).
            uint32_t dlo[8], dhi[8];
            static_for<0, 8>([&](auto mI) {
                constexpr int m = decltype(mI)::value;
                const uint32_t j = (uint32_t)(lane + 64 * m);
                const uint32_t tt = (j - a) & (uint32_t)(2 * FN - 1);
                const uint32_t quad = tt / FH;
                const uint2 rr = acc[c][tt & (uint32_t)(FH - 1)];
                const uint2 pl = acc[c][j];
                const uint32_t f = (quad & 1u) ? rr.y : rr.x, sc = (quad & 1u) ? rr.x : rr.y;
                const uint32_t v0 = (quad == 2u || quad == 3u) ? 0u - f : f;
                const uint32_t v1 = (quad == 1u || quad == 2u) ? 0u - sc : sc;
                dlo[m] = (v0 - pl.x + kDigitOffset) ^ kDigitSignBits;
                dhi[m] = (v1 - pl.y + kDigitOffset) ^ kDigitSignBits;
            });
#pragma unroll 1
            for (int jj = 0; jj < 3; ++jj) {
                const int p = 3 * c + jj;
                __syncthreads();   // every wave is done with the previous key stage
                static_for<0, F_PRE>([&](auto kI) { kst[tid + decltype(kI)::value * F_THREADS] = pre[decltype(kI)::value]; });
                {
                    int ni = i, np = p + 1;
                    if (np == 6) {
                        np = 0;
                        ++ni;
                    }
                    if (ni >= n) ni = 0;   // past the last step: reload step 0 (unused)
                    const d2 *src = spec + ((int64_t)ni * 6 + np) * STAGE_D2;
                    static_for<0, F_PRE>([&](auto kI) { pre[decltype(kI)::value] = src[tid + decltype(kI)::value * F_THREADS]; });
                }
                __syncthreads();   // stage visible
                if (wave >= FG / 2) __builtin_amdgcn_s_setprio(1);   // issue balance, first half

                const uint32_t sh = (uint32_t)(32 - 7 * (jj + 1));
                d2 x[8];
                static_for<0, 8>([&](auto mI) {
                    constexpr int m = decltype(mI)::value;
                    const double lo = (double)sbfe7(dlo[m], sh);
                    const double hi = (double)sbfe7(dhi[m], sh);
                    x[m] = cmul(d2{lo, hi}, twist_slot(m));
                });
                __builtin_amdgcn_sched_barrier(0);
                fft_fwd<true>(x, scr, lane, t);
                __builtin_amdgcn_sched_barrier(0);
                if (wave >= FG / 2) __builtin_amdgcn_s_setprio(1);   // issue balance, first half
                static_for<0, 8>([&](auto sI) {
                    constexpr int sl = decltype(sI)::value;
                    outA[sl] = cmac(outA[sl], x[sl], kst[sl * 64 + lane]);
                    outB[sl] = cmac(outB[sl], x[sl], kst[FH + sl * 64 + lane]);
                    if constexpr (sl == 3) __builtin_amdgcn_s_setprio(0);
                });
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        // inverse transforms, untwist, round, accumulate (this wave's ACC only)
        wave_lds_fence();
        auto finish = [&](d2 (&x)[8], uint2 *dst) {
            fft_inv(x, scr, lane, t);
            static_for<0, 8>([&](auto mI) {
                constexpr int m = decltype(mI)::value;
                const d2 y = cmul(x[m], cconj(twist_slot(m)));
                const int j = lane + 64 * m;
                uint2 v = dst[j];
                v.x += round_mod32(y.x);
                v.y += round_mod32(y.y);
                dst[j] = v;
            });
        };
        if (wave >= FG / 2) __builtin_amdgcn_s_setprio(1);   // issue balance, first inverse
        finish(outA, acc[0]);
        __builtin_amdgcn_s_setprio(0);
        __builtin_amdgcn_sched_barrier(0);
        finish(outB, acc[1]);
        wave_lds_fence();
    }

    // sample extraction
    if (live) {
        uint32_t *e = ext + g * (FN + 1);
        auto coef = [&](int q, int k) { return k < FH ? acc[q][k].x : acc[q][k - FH].y; };
        for (int j = lane; j <= FN; j += 64) {
            uint32_t v;
            if (j == 0) v = coef(0, 0);
            else if (j == FN) v = coef(1, 0);
            else v = 0u - coef(0, FN - j);
            e[j] = v;
        }
    }
}

}  // namespace

int br_fft_batch_ok(const cemu_cloud_key *ck, int64_t B)
{
    // one workgroup per gate (latency kernel) or per FG gates
    const int fg = ck->tuning.fft_gates_per_wg;
    const int64_t items = fg == 1 ? B * 64 * LAT_WAVES : (B + fg - 1) / fg * 64 * fg;
    if (B < 0 || items > (int64_t)0xffffffff) return fail(CEMU_ERR_RANGE, "batch too large for one launch of this shape");
    return CEMU_OK;
}

int build_bk_fft(cemu_cloud_key *ck, hipStream_t s)
{
    if (ck->p.N != FN) return fail(CEMU_ERR_UNSUPPORTED, "the FFT64 form is built for N = 1024");
    if (ck->d_bkfft) return CEMU_OK;
    const size_t polys = (size_t)ck->p.n * 6 * 2;
    if (hipMalloc(&ck->d_bkfft, polys * FH * sizeof(d2)) != hipSuccess)
        return fail(CEMU_ERR_OOM, "device allocation (FFT key) failed");
    hipLaunchKernelGGL(bk_fft_prepare_kernel, dim3((unsigned)polys), dim3(64), 0, s, ck->d_bk8,
                       reinterpret_cast<d2 *>(ck->d_bkfft));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(CEMU_ERR_HIP, std::string("bk_fft_prepare launch: ") + hipGetErrorString(e));
    return CEMU_OK;
}

int launch_br_fft(cemu_cloud_key *ck, const uint16_t *bars, int64_t B, uint32_t *ext, hipStream_t s)
{
    if (ck->p.N != FN) return fail(CEMU_ERR_UNSUPPORTED, "the FFT64 form is built for N = 1024");
    const int n = ck->p.n;
    if (const int rc = build_bk_fft(ck, s)) return rc;   // normally done at key generation
    if (const int rc = br_fft_batch_ok(ck, B)) return rc;
    const int fg = ck->tuning.fft_gates_per_wg;
    const d2 *spec = reinterpret_cast<const d2 *>(ck->d_bkfft);
    if (B == 0) return CEMU_OK;
    auto launch = [&](int shape, const uint16_t *b, int64_t cnt, uint32_t *x) {
        if (shape == 1)
            launch_br_fft_lat(reinterpret_cast<const double *>(spec), b, n, cnt, x, s);
        else if (shape == 4)
            hipLaunchKernelGGL(br_fft_kernel<4>, dim3((unsigned)((cnt + 3) / 4)), dim3(256), 0, s, spec, b, n, cnt, x);
        else
            hipLaunchKernelGGL(br_fft_kernel<8>, dim3((unsigned)((cnt + 7) / 8)), dim3(512), 0, s, spec, b, n, cnt, x);
    };
    // Every shape runs one workgroup per CU, so a launch proceeds in rounds of
    // fg * CUs gates, and a round costs the same however few of its
    // workgroups are busy. A batch of k full rounds plus a short tail r runs
    // the tail as its own launch of a smaller shape whenever that is cheaper
    // than one more round. Measured round times on MI355X (630 steps):
    // latency kernel (CUs gates) 2.54 ms, 4 gates per workgroup 8.8 ms,
    // 8 gates per workgroup 10.8 ms; so a tail of up to 3 CUs gates goes to
    // the latency kernel, and behind 8-gate rounds one of up to 4 CUs gates
    // to the 4-gate shape. Outputs do not depend on the shape.
    const int64_t cus = ck->num_cus;
    int64_t full = B;
    int tail_shape = 0;
    if (cus > 0 && fg > 1) {
        const int64_t round = fg * cus;
        const int64_t r = B % round;
        if (B >= round && r > 0) {
            if (r <= 3 * cus) tail_shape = 1;
            else if (fg == 8 && r <= 4 * cus) tail_shape = 4;
            if (tail_shape) full = B - r;
        }
    }
    launch(fg, bars, full, ext);
    if (tail_shape) launch(tail_shape, bars + full * (int64_t)(n + 1), B - full, ext + full * (int64_t)(FN + 1));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(CEMU_ERR_HIP, std::string("br_fft_kernel launch: ") + hipGetErrorString(e));
    return CEMU_OK;
}

}  // namespace cemu
