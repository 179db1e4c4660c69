// Shared device code of the FP64-FFT blind-rotation kernels (gfx950): the
// negacyclic transform, its twiddles and transposes, and the constants of
// the digit decomposition. Included by cemu_br_fft.hip (key preparation and
// throughput kernel) and cemu_br_fft_lat.hip (latency kernel); every
// definition has internal linkage.
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
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

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

constexpr int FN = 1024;          // ring degree handled by these kernels
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
// default issue priority after the first transpose (see br_fft_kernel in cemu_br_fft.hip).
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

constexpr int STAGE_D2 = 2 * FH;   // key spectra of one digit row: (q, slot, lane)
constexpr int LAT_WAVES = 8;       // latency kernel: six digit-row waves and two inverse waves; all eight reduce

}  // namespace
}  // namespace cemu
