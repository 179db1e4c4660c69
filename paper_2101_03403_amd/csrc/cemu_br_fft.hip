// Blind rotation with FP64 negacyclic-FFT products (gfx950).
//
// Negacyclic product in R[X]/(X^N+1), N = 1024, through a length-N/2 complex
// FFT: since X^N + 1 = (X^{N/2} - i)(X^{N/2} + i) and the polynomials are
// real, P is determined by P mod (X^{N/2} - i) = sum_{j<N/2} (P_j + i P_{j+N/2}) X^j.
// Substituting X = w Y with w = exp(i pi / N) (so w^{N/2} = i) turns that
// ring into C[Y]/(Y^{N/2} - 1), where products are cyclic convolutions:
//   z_j = (P_j + i P_{j+N/2}) w^j  ->  FFT_{N/2}  ->  pointwise products
//   ->  inverse FFT / (N/2)  ->  times w^{-j}  ->  (R_j, R_{j+N/2}) = (Re, Im).
// The key polynomials are taken as centred int32 values and their spectra
// are precomputed once per key; digits are small integers. Every product is
// an integer polynomial, so the double result rounds to the exact integer as
// long as the transform error stays below 1/2. Sums stay near 2^42 for the
// random key coefficients (3 * 2^50 is the adversarial bound), where the
// error is far below 1/2; but the form is not exact by construction, unlike
// the int8 form, and its deviation is measured against the oracle.
//
// FFT of 512 points per wave: lane l holds x[l + 64 m], m = 0..7. Three
// radix-8 passes (512 = 8^3, decimation in frequency) with two LDS
// transposes between them; the spectrum ends up with lane 8 k0 + k1 holding
// X[k0 + 8 k1 + 64 k2] in slot k2, and the inverse runs the passes backwards
// from that order, so no bit reversal is ever done. Key spectra are stored in
// the same (slot, lane) order.
//
// Throughput kernel: one wave per gate, FG = 8 (default) or 4 gates per
// workgroup: each wave keeps its accumulator (2 x N u32, as 8-byte records of
// the coefficient pair (j, j + N/2)) and its FFT transpose scratch in LDS; the
// key spectra of one digit row (16 KiB) are staged in LDS once per workgroup,
// prefetched through registers one row ahead.
//
// Latency kernel (narrow batches): one gate per workgroup of 8 waves. Six
// waves, one per gadget digit, run the 6 forward transforms of a step side
// by side and leave their spectra in LDS; every wave then forms, for one
// frequency slot, both outputs' sums over the six rows (in a fixed row
// order, its key values prefetched into registers a step ahead), and two
// waves run the two inverse transforms. A step then costs about three
// transform latencies instead of eight.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "cemu_kernels.h"

namespace cemu {
namespace {

typedef double d2 __attribute__((ext_vector_type(2)));

template <int B, int E, class F>
__device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

constexpr int FN = 1024;          // ring degree handled by this kernel
constexpr int FH = FN / 2;        // complex FFT length
constexpr int SCR = 8 * 72;       // transpose scratch entries per wave (8 blocks of 64 + pad 8)
constexpr uint32_t kDigitOffset = 0x81020400u;   // see cemu_br_int8.hip
// Top bit of each 7-bit digit field (bits 31, 24, 17). With the offset added,
// a field holds d + 64 for the signed digit d in [-64, 64); flipping its top
// bit leaves d in 7-bit two's complement, so a signed bit-field extract
// yields d itself.
constexpr uint32_t kDigitSignBits = 0x81020000u;

__device__ __forceinline__ d2 cmul(d2 a, d2 b) { return d2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ __forceinline__ d2 cconj(d2 a) { return d2{a.x, -a.y}; }
// acc + a * b as four fused multiply-adds (written out: the compiler does not
// fold the accumulate into the multiply's own fused operations, and would
// spend two multiplies, two fused operations and two adds).
__device__ __forceinline__ d2 cmac(d2 acc, d2 a, d2 b)
{
    return d2{fma(-a.y, b.y, fma(a.x, b.x, acc.x)), fma(a.y, b.x, fma(a.x, b.y, acc.y))};
}

// Nearest integer of y reduced mod 2^32, for |y| < 2^51: adding 1.5 * 2^52
// lands in the binade [2^52, 2^53) whose spacing is 1, so the addition itself
// rounds (to nearest, ties to even, as rint does) and the low mantissa bits
// hold 2^51 + rint(y), whose low 32 bits are rint(y) mod 2^32. One FP64 add
// instead of rint plus a double -> int64 conversion. The bound holds with a
// wide margin: |y| <= 6 * N * 64 * 2^31 only for adversarial keys, and the
// centred random key coefficients keep sums near 2^42.
__device__ __forceinline__ uint32_t round_mod32(double y)
{
    return (uint32_t)__double_as_longlong(y + 6755399441055744.0);
}

__device__ __forceinline__ d2 cexp_unit(double theta)
{
    double s, c;
    sincos(theta, &s, &c);
    return d2{c, s};
}

// In-register DFT of length 8 over x[0..7]; INV selects the +i sign.
// Radix-2 split into even and odd outputs; the sqrt(1/2) factors of the odd
// quarter are applied by the final fused multiply-adds (52 FP64 operations).
template <bool INV>
__device__ __forceinline__ void dft8(d2 (&x)[8])
{
    const double r = 0.70710678118654752440;
    const d2 a0 = x[0] + x[4], a4 = x[0] - x[4];
    const d2 a1 = x[1] + x[5], a5 = x[1] - x[5];
    const d2 a2 = x[2] + x[6], a6 = x[2] - x[6];
    const d2 a3 = x[3] + x[7], a7 = x[3] - x[7];
    double s1, s2, w1, w2;
    d2 a6r;
    if constexpr (!INV) {
        const double u1 = a5.x + a5.y, u2 = a5.y - a5.x, v1 = a7.y - a7.x, v2 = a7.x + a7.y;
        s1 = u1 + v1; s2 = u2 - v2; w1 = u2 + v2; w2 = v1 - u1;
        a6r = d2{a6.y, -a6.x};                              // * -i
    } else {
        const double u1 = a5.x - a5.y, u2 = a5.x + a5.y, v1 = a7.x + a7.y, v2 = a7.x - a7.y;
        s1 = u1 - v1; s2 = u2 + v2; w1 = v2 - u2; w2 = u1 + v1;
        a6r = d2{-a6.y, a6.x};                              // * i
    }
    const d2 b0 = a0 + a2, b2 = a0 - a2, b1 = a1 + a3;
    const d2 b4 = a4 + a6r, b6 = a4 - a6r;
    d2 b3 = a1 - a3;
    if constexpr (!INV) b3 = d2{b3.y, -b3.x};
    else b3 = d2{-b3.y, b3.x};
    x[0] = b0 + b1;
    x[4] = b0 - b1;
    x[2] = b2 + b3;
    x[6] = b2 - b3;
    x[1] = d2{fma(r, s1, b4.x), fma(r, s2, b4.y)};
    x[5] = d2{fma(-r, s1, b4.x), fma(-r, s2, b4.y)};
    x[3] = d2{fma(r, w1, b6.x), fma(r, w2, b6.y)};
    x[7] = d2{fma(-r, w1, b6.x), fma(-r, w2, b6.y)};
}

// x[s] *= b^s for s = 1..7.
__device__ __forceinline__ void twiddle_pow(d2 (&x)[8], d2 b)
{
    d2 w = b;
#pragma unroll
    for (int s = 1; s < 8; ++s) {
        x[s] = cmul(x[s], w);
        if (s < 7) w = cmul(w, b);
    }
}

// x[s] *= c * b^s for s = 0..7.
__device__ __forceinline__ void twiddle_pow(d2 (&x)[8], d2 c, d2 b)
{
    d2 w = c;
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        x[s] = cmul(x[s], w);
        if (s < 7) w = cmul(w, b);
    }
}

// Slot/lane transposes through the wave's scratch, hi = lane>>3, lo = lane&7.
// Both maps are involutions:
//   xpose_lo: out(hi, lo; s) = in(hi, s; lo)   (exchange lo with the slot)
//   xpose_hi: out(hi, lo; s) = in(s, lo; hi)   (exchange hi with the slot)
// Entry positions are a per-lane base plus a per-slot constant, and every
// 16-lane group of an access hits 16 distinct 4-bank groups (72 = 8 mod 16
// separates the two hi values of a group; 9 lo mod 16 is injective on 0..7).
// The scratch is private to the wave and LDS operations of one wave execute
// in order, so a wavefront-scope fence (compiler ordering only) suffices.
__device__ __forceinline__ void wave_lds_fence() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); }

__device__ __forceinline__ void xpose_lo(d2 (&x)[8], d2 *scr, int lane)
{
    const int hi = lane >> 3, lo = lane & 7;
    d2 *w = scr + 72 * hi + lo;          // entry (hi, a = s, b = lo): 72 hi + 9 s + lo
    d2 *r = scr + 72 * hi + 9 * lo;      // entry (hi, a = lo, b = s): 72 hi + 9 lo + s
#pragma unroll
    for (int s = 0; s < 8; ++s) w[9 * s] = x[s];
    wave_lds_fence();
#pragma unroll
    for (int s = 0; s < 8; ++s) x[s] = r[s];
    wave_lds_fence();
}

__device__ __forceinline__ void xpose_hi(d2 (&x)[8], d2 *scr, int lane)
{
    const int hi = lane >> 3, lo = lane & 7;
    d2 *w = scr + lane;                  // entry (a = s, b = hi, lo): 72 s + 8 hi + lo
    d2 *r = scr + 72 * hi + lo;          // entry (a = hi, b = s, lo): 72 hi + 8 s + lo
#pragma unroll
    for (int s = 0; s < 8; ++s) w[72 * s] = x[s];
    wave_lds_fence();
#pragma unroll
    for (int s = 0; s < 8; ++s) x[s] = r[8 * s];
    wave_lds_fence();
}

// Twiddle bases of one lane (W = exp(-2 pi i / 512)).
struct Tw {
    d2 tw;    // w^lane, w = exp(i pi / N): the per-lane part of the twist
    d2 f1;    // W^lane                       (forward pass 1, powers over slot)
    d2 f2;    // W^(8 (lane & 7))             (forward pass 2; conj for inverse pass 1)
    d2 i2c;   // W^-((lane & 7) (lane >> 3)) w^-(lane & 7) / (N/2)  (inverse pass 2 constant, with untwist part and scale)
    d2 i2b;   // W^-(8 (lane >> 3)) w^-8        (inverse pass 2, power base)
};

// Hide a value's provenance from the optimiser so that products of it
// (twiddle and twist powers) are recomputed where they are used instead of
// being hoisted out of the step loop: hoisting them all would overflow the
// 256 registers a wave has at two waves per SIMD.
__device__ __forceinline__ void launder(d2 &v)
{
    double a = v.x, b = v.y;
    asm volatile("" : "+v"(a), "+v"(b));
    v = d2{a, b};
}

__device__ __forceinline__ Tw make_tw(int lane)
{
    const double two_pi_over = -2.0 * 3.14159265358979323846 / FH;
    Tw t;
    t.f1 = cexp_unit(two_pi_over * lane);
    t.f2 = cexp_unit(two_pi_over * (8 * (lane & 7)));
    t.tw = cexp_unit(3.14159265358979323846 / FN * lane);
    // the untwist w^-(8 j1 + j0) of the destination lane (j1, j0) after the
    // following transpose = w^-j0 * (w^-8)^j1: a power series in the slot j1
    t.i2c = cmul(cexp_unit(-two_pi_over * ((lane & 7) * (lane >> 3))),
                 cexp_unit(-3.14159265358979323846 / FN * (lane & 7))) * (1.0 / FH);
    t.i2b = cmul(cexp_unit(-two_pi_over * (8 * (lane >> 3))), cexp_unit(-3.14159265358979323846 / FN * 8));
    return t;
}

// Forward twisted FFT_512: in x[m] = P-fold[lane + 64 m] * w^(64 m) (the
// per-slot part of the twist); the per-lane part w^lane commutes with the
// first length-8 DFT and is applied with its twiddles. Out: slot k2 of lane
// 8 k0 + k1 = Z[k0 + 8 k1 + 64 k2]. DROP_PRIO: return the wave to the
// default issue priority after the first transpose (see br_fft_kernel).
template <bool DROP_PRIO = false>
__device__ __forceinline__ void fft_fwd(d2 (&x)[8], d2 *scr, int lane, const Tw &t)
{
    dft8<false>(x);                 // lane (j1, j0): over j2 -> k0
    twiddle_pow(x, t.tw, t.f1);     // w^lane * W^((8 j1 + j0) k0): twist (per-lane part) + twiddle
    xpose_hi(x, scr, lane);         // lane (k0, j0), slot j1
    if constexpr (DROP_PRIO) __builtin_amdgcn_s_setprio(0);
    __builtin_amdgcn_sched_barrier(0);
    dft8<false>(x);                 // over j1 -> k1
    twiddle_pow(x, t.f2);           // W^(8 j0 k1)
    xpose_lo(x, scr, lane);         // lane (k0, k1), slot j0
    __builtin_amdgcn_sched_barrier(0);
    dft8<false>(x);                 // over j0 -> k2
}

// Inverse: the data movement of fft_fwd run backwards; the per-lane untwist
// w^-lane and the 1/(N/2) scale ride on the last twiddle (they commute with the
// final length-8 DFT); the caller multiplies slot m by conj(w^(64 m)).
__device__ __forceinline__ void fft_inv(d2 (&x)[8], d2 *scr, int lane, const Tw &t)
{
    dft8<true>(x);                  // lane (k0, k1): over k2 -> j0
    twiddle_pow(x, cconj(t.f2));    // W^-(8 k1 j0)
    xpose_lo(x, scr, lane);         // lane (k0, j0), slot k1
    __builtin_amdgcn_sched_barrier(0);
    dft8<true>(x);                  // over k1 -> j1
    twiddle_pow(x, t.i2c, t.i2b);   // W^-((8 j1 + j0) k0)
    xpose_hi(x, scr, lane);         // lane (j1, j0), slot k0
    __builtin_amdgcn_sched_barrier(0);
    dft8<true>(x);                  // over k0 -> j2
}

// exp(i pi m / 16), m = 0..7: the twist w^(64 m) of slot m.
__device__ __forceinline__ d2 twist_slot(int m)
{
    const double c[8] = {1.0, 0.98078528040323044913, 0.92387953251128675613, 0.83146961230254523708,
                         0.70710678118654752440, 0.55557023301960222474, 0.38268343236508977173,
                         0.19509032201612826785};
    return d2{c[m], c[(8 - m) & 7] * (m ? 1.0 : 0.0)};
}

// Signed 7-bit field of x at bit offset off (wave-uniform), sign-extended:
// one v_bfe_i32. Written as a VALU instruction because the compiler's own
// signed bit-field-extract builtin was followed by an unsigned conversion to
// double here (the sign was lost).
__device__ __forceinline__ int32_t sbfe7(uint32_t x, uint32_t off)
{
    int32_t r;
    asm("v_bfe_i32 %0, %1, %2, 7" : "=v"(r) : "v"(x), "s"(off));
    return r;
}

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

constexpr int STAGE_D2 = 2 * FH;           // key spectra of one digit row: (q, slot, lane)

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

constexpr int LAT_WAVES = 8;   // six digit-row waves and two inverse waves; all eight reduce

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
            hipLaunchKernelGGL(br_fft_lat_kernel, dim3((unsigned)cnt), dim3(64 * LAT_WAVES), 0, s, spec, b, n, x);
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
