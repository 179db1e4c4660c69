// Launchers of the blind-rotation kernels (one translation unit per form).
#pragma once

#include <hip/hip_runtime.h>

#include "cemu_internal.h"

namespace cemu {

// Blind rotation + sample extraction for B mod-switched samples.
//   bars: device u16 [B][n+1] (abar_0 .. abar_{n-1}, bbar), values in [0, 2N)
//   ext:  device u32 [B][N+1] extracted samples
int launch_br_int8(const cemu_cloud_key *ck, const uint16_t *bars, int64_t B, uint32_t *ext, hipStream_t s);
int launch_br_fft(cemu_cloud_key *ck, const uint16_t *bars, int64_t B, uint32_t *ext, hipStream_t s);

// The FFT form of the bootstrapping key (ck->d_bkfft), allocated and computed
// on stream s if it is not there yet; N = 1024 only.
int build_bk_fft(cemu_cloud_key *ck, hipStream_t s);

// One launch of the FFT latency kernel (one gate per workgroup of
// 64 * LAT_WAVES threads) for cnt gates; spec is the key in the FFT form
// (ck->d_bkfft). Errors are left to hipGetLastError.
void launch_br_fft_lat(const double *spec, const uint16_t *bars, int32_t n, int64_t cnt, uint32_t *ext,
                       hipStream_t s);

// CEMU_OK if one launch of the key's current shape for the form holds B
// blind rotations (a dispatch counts at most 2^32 - 1 work-items), else
// CEMU_ERR_RANGE with the message set. The launchers check it too.
int br_int8_batch_ok(const cemu_cloud_key *ck, int64_t B);
int br_fft_batch_ok(const cemu_cloud_key *ck, int64_t B);

// Key switching of B extracted samples as an int8 MFMA contraction; output
// row io[g] (or g) of out. Requires ks_mfma_supported(ck->p).
int launch_ks_mfma(const cemu_cloud_key *ck, const uint32_t *ext, const int32_t *io, uint32_t *out, int64_t B,
                   hipStream_t s);

}  // namespace cemu
