/*
 * cemu.h -- C ABI of the MI355X (gfx950) batched TFHE gate-bootstrapping
 * library that runs the hot path under CryptoEmu's homomorphic functional
 * units (Gong and Negrut, "CryptoEmu: An Instruction Set Emulator for
 * Computation Over Ciphers", arXiv 2101.03403).
 *
 * The paper builds every functional unit (adder, subtractor, shifters,
 * multiplier, divider, bitwise units, Sec. 5-6) from bootstrapped binary
 * gates of the TFHE library and names bootstrapping the dominant cost (Sec. 3,
 * Table "TFHEbenchmark"). Its API surface -- secret/cloud keyset generation,
 * encryption and decryption with the secret keyset, gate evaluation with the
 * cloud keyset, and the unbootstrapped CONSTANT / NOT / COPY (Sec. 3) -- is the
 * surface exported here, with gate evaluation batched over many gates.
 *
 * Conventions shared by every entry point:
 *  - Torus elements are uint32_t (T = R/Z represented by Z/2^32, wraparound).
 *  - An LWE ciphertext of dimension d is d+1 consecutive uint32_t words
 *    [a_0 .. a_{d-1}, b]; batches are ciphertext-major, densely packed.
 *  - Bits are encoded as +1/8 (true) and -1/8 (false).
 *  - Pointers documented "device" must be device memory of the GPU on which
 *    the cloud key was created, 4-byte aligned; "host" pointers are ordinary
 *    host memory. All batch buffers are caller-owned; the library never frees
 *    them and never keeps them after the call returns (device calls only
 *    enqueue work on the caller's stream).
 *  - Keys are opaque handles owned by the library until cemu_free_*.
 *  - Device entry points enqueue on the given hipStream_t (passed as void*,
 *    NULL = the default stream) and return without synchronising.
 *  - Return value: CEMU_OK (0) or a negative cemu_status. Nothing throws or
 *    aborts across the ABI. cemu_last_error() returns a description of the
 *    last failure of the calling thread.
 */
#ifndef CEMU_H
#define CEMU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum cemu_status {
    CEMU_OK = 0,
    CEMU_ERR_PARAM = -1,        /* invalid or unsupported parameter value      */
    CEMU_ERR_NULL = -2,         /* required pointer is NULL                     */
    CEMU_ERR_ALIGN = -3,        /* pointer not 4-byte aligned                   */
    CEMU_ERR_OOM = -4,          /* host or device allocation failed             */
    CEMU_ERR_HIP = -5,          /* HIP runtime error                            */
    CEMU_ERR_UNSUPPORTED = -6,  /* parameter set the kernels cannot run         */
    CEMU_ERR_OP = -7,           /* reserved: op codes are not checked on the device */
    CEMU_ERR_RANGE = -8         /* index or size out of range                   */
} cemu_status;

/* Parameter sets. CEMU_STD is the standard 80-bit TFHE gate-bootstrapping set
 * (n = 630, N = 1024, k = 1, l = 3, Bgbit = 7, t = 8, basebit = 2, LWE and
 * key-switching noise 2^-15, bootstrapping-key noise 2^-25). CEMU_TOY is an
 * insecure test set (n = 256, N = 512, same other values). */
enum { CEMU_STD = 0, CEMU_TOY = 1 };

/* Forms of the negacyclic polynomial products inside the blind rotation.
 * CEMU_FORM_INT8: each key coefficient split into four signed 8-bit limbs,
 *   products on int8 MFMA with int32 accumulation; exact modulo 2^32.
 * CEMU_FORM_FFT64: twisted negacyclic FFT in IEEE double per product; the
 *   result is rounded to the nearest integer and can differ from the exact
 *   product in the low bits. */
enum { CEMU_FORM_INT8 = 0, CEMU_FORM_FFT64 = 1 };

/* Bootstrapped binary gate op codes (the ten gates of Table "TFHEbenchmark").
 * With inputs a (first) and b (second):
 *   NAND, AND, OR, XOR, XNOR, NOR, ANDNY = (not a) and b, ANDYN = a and (not b),
 *   ORNY = (not a) or b, ORYN = a or (not b). */
enum {
    CEMU_NAND = 0, CEMU_AND = 1, CEMU_OR = 2, CEMU_XOR = 3, CEMU_XNOR = 4,
    CEMU_NOR = 5, CEMU_ANDNY = 6, CEMU_ANDYN = 7, CEMU_ORNY = 8, CEMU_ORYN = 9,
    CEMU_NUM_GATE_OPS = 10
};

/* Largest LWE dimension of the unbootstrapped row operations (NOT, COPY,
 * CONSTANT), and of keys: the key switch computes the n + 1 output words of
 * a sample in one workgroup pass of at most 768 columns. */
#define CEMU_MAX_LWE_N 4096
#define CEMU_MAX_KEY_N 767

typedef struct cemu_params {
    int32_t n;         /* LWE dimension of gate ciphertexts: 1..CEMU_MAX_KEY_N */
    int32_t N;         /* TRLWE ring degree: 512 or 1024                      */
    int32_t k;         /* TRLWE mask count: must be 1                        */
    int32_t l;         /* bootstrapping-key gadget length: must be 3          */
    int32_t bgbit;     /* log2 gadget base: must be 7 (digits in [-64, 64))  */
    int32_t t;         /* key-switching length: 1..16, t*basebit <= 32       */
    int32_t basebit;   /* key-switching base bits: must be 2                  */
    int32_t reserved;  /* set to 0                                           */
    double sigma_lwe;  /* std dev of fresh LWE noise, torus units, in [0, 1] */
    double sigma_ks;   /* std dev of key-switching-key noise, same range     */
    double sigma_bk;   /* std dev of bootstrapping-key noise, same range     */
} cemu_params;

typedef struct cemu_secret_key cemu_secret_key;
typedef struct cemu_cloud_key cemu_cloud_key;

/* Fill *p with a named parameter set (CEMU_STD or CEMU_TOY).
 * Errors: CEMU_ERR_NULL, CEMU_ERR_PARAM (unknown set). */
int cemu_params_default(cemu_params *p, int which);

/* Secret-keyset and cloud-keyset generation (Sec. 3, "TFHE API": keyset
 * generation precedes all gate evaluation). Deterministic in seed: every
 * random value is a Philox4x32-10 output at a fixed counter, keyed by seed,
 * so the same seed gives the same keys on any machine. The secret key stays
 * on the host. The cloud key (bootstrapping key in the int8-limb layout and
 * the key-switching key) is uploaded to the current HIP device; for N = 1024
 * the FFT form of the bootstrapping key is built there too, before the call
 * returns, so that later gate calls need no set-up.
 * Ownership: *sk and *ck are owned by the library until cemu_free_*.
 * Errors: CEMU_ERR_NULL, CEMU_ERR_PARAM / CEMU_ERR_UNSUPPORTED (parameter set
 * outside the limits stated in cemu_params), CEMU_ERR_OOM, CEMU_ERR_HIP. */
int cemu_keygen(const cemu_params *p, uint64_t seed, cemu_secret_key **sk, cemu_cloud_key **ck);

/* Copy the parameters of a key. */
int cemu_secret_params(const cemu_secret_key *sk, cemu_params *p);
int cemu_cloud_params(const cemu_cloud_key *ck, cemu_params *p);

/* Encrypt (Sec. 3, Table "TFHEbenchmark": Encrypt). bits: host [count]
 * (0 = false, nonzero = true). out: host [count][n+1]. Ciphertext e uses the
 * encryption stream (seed, first_index + e), so a batch can be produced in
 * pieces. Errors: CEMU_ERR_NULL, CEMU_ERR_RANGE (count < 0). */
int cemu_encrypt(const cemu_secret_key *sk, const uint8_t *bits, int64_t count, uint64_t seed,
                 uint64_t first_index, uint32_t *out);

/* Decrypt (Table "TFHEbenchmark": Decrypt): bit = (phase as int32) > 0.
 * ct: host [count][n+1]; bits: host [count].
 * cemu_decrypt_extracted takes dimension-N samples [count][N+1] (the output
 * of cemu_blind_rotate_extract), decrypted with the TRLWE key coefficients.
 * Errors: CEMU_ERR_NULL, CEMU_ERR_RANGE. */
int cemu_decrypt(const cemu_secret_key *sk, const uint32_t *ct, int64_t count, uint8_t *bits);
int cemu_decrypt_extracted(const cemu_secret_key *sk, const uint32_t *ct, int64_t count, uint8_t *bits);

/* Phase b - <a, s> of each ciphertext, for noise measurement. extracted = 0:
 * ct is [count][n+1] under the LWE key; extracted = 1: [count][N+1] under the
 * TRLWE key coefficients. phase: host [count]. */
int cemu_phase(const cemu_secret_key *sk, int extracted, const uint32_t *ct, int64_t count, uint32_t *phase);

/* Batched bootstrapped binary gates: lincomb + modulus switch + blind
 * rotation + sample extraction + key switching, for B independent gates.
 * The paper evaluates each gate as one call of the TFHE library (Sec. 3,
 * Table "TFHEbenchmark"; correctness f(a, b) = Dec(g(Enc a, Enc b)), Sec. 2)
 * and does not spell out its steps; they are read as TFHE's gate
 * bootstrapping, which the paper builds on:
 *   1. c = (0, ..., 0, kappa) + w1 c1 + w2 c2 with the gate's constants
 *      (NAND +1/8, -1, -1; AND -1/8, 1, 1; OR +1/8, 1, 1; XOR +1/4, 2, 2;
 *      XNOR -1/4, -2, -2; NOR -1/8, -1, -1; ANDNY -1/8, -1, 1; ANDYN -1/8,
 *      1, -1; ORNY +1/8, -1, 1; ORYN +1/8, 1, -1);
 *   2. every word rescaled to Z/2N: nearest integer of x 2N / 2^32, ties up,
 *      2N wrapping to 0;
 *   3. blind rotation: ACC = (0, X^-bbar v) with v = sum_j (1/8) X^j, then
 *      for each i with abar_i != 0, ACC += BK_i (external product)
 *      (X^abar_i ACC - ACC), the difference decomposed into l = 3 signed
 *      digits of Bgbit = 7 bits (rounded to 21 bits, ties up, digits in
 *      [-64, 64));
 *   4. sample extraction of coefficient 0: (A_0, -A_{N-1}, ..., -A_1, B_0);
 *   5. key switching as cemu_key_switch.
 * The output encrypts g(a, b) as +-1/8 under the LWE key.
 *   ops:      device uint8_t [B], gate op codes (CEMU_NAND .. CEMU_ORYN)
 *   pool_in:  device uint32_t [P_in][n+1], ciphertext pool read by the gates
 *   ia, ib:   device int32_t [B], row of the first / second input in pool_in
 *   io:       device int32_t [B], row of pool_out receiving gate g's output
 *             (rows distinct within the batch); NULL means row g
 *   pool_out: device uint32_t [P_out][n+1]; may alias pool_in only if no
 *             output row is also an input row of this batch
 * Row indices are not range-checked on the device: the caller guarantees
 * 0 <= ia, ib < P_in and io (or g) < P_out, and unknown op codes produce an
 * unspecified ciphertext. B = 0 is a no-op. Scratch: the library keeps
 * per-cloud-key device workspaces sized for the largest B seen (allocated on
 * demand, so this call may allocate). Calls sharing one cloud key must not
 * overlap in time on different streams. A hipGraph captured around these
 * calls records the workspace addresses: size the workspaces first (run the
 * same launches once eagerly), and replay the graph only while no later call
 * on the same cloud key has needed a larger workspace (that reallocates it).
 * Errors: CEMU_ERR_NULL, CEMU_ERR_ALIGN, CEMU_ERR_RANGE (B < 0, B > 2^40,
 * or more gates than one launch of the selected blind-rotation shape holds:
 * a dispatch counts at most 2^32 - 1 work-items, i.e. 11.1M gates for the
 * latency kernel, 67.1M for the FFT throughput kernels and 134M (8 waves) or
 * 268M (4 waves) for the int8 form), CEMU_ERR_PARAM (unknown form), CEMU_ERR_UNSUPPORTED (FFT64 form with
 * N != 1024: it is built for the standard ring degree only), CEMU_ERR_OOM,
 * CEMU_ERR_HIP. */
int cemu_bootstrap_gates(const cemu_cloud_key *ck, int form, const uint8_t *ops, const uint32_t *pool_in,
                         const int32_t *ia, const int32_t *ib, const int32_t *io, uint32_t *pool_out,
                         int64_t B, void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * gates as cemu_bootstrap_gates, same arguments and the same outputs bit for
 * bit, with no hipMalloc, hipFree or other allocation in the call. The
 * workspace is a fixed scratch array in the library's device code (22 MiB
 * on each GPU the library runs on, held until the process ends; its address
 * is looked up at key generation), so B is limited to
 * CEMU_NOALLOC_MAX_GATES. Every call on one GPU shares that one array:
 * calls whose work overlaps in time on the same GPU (several streams or host
 * threads, any cloud keys) race and produce wrong ciphertexts, so serialise
 * them, e.g. on one stream. Each call writes every scratch word it reads, so
 * nothing carries over from the previous call. Kernel timing
 * (cemu_profile_enable) records nothing for this entry point.
 * Errors: as cemu_bootstrap_gates, plus CEMU_ERR_RANGE for
 * B > CEMU_NOALLOC_MAX_GATES. */
#define CEMU_NOALLOC_MAX_GATES 4096
int cemu_bootstrap_gates_noalloc(const cemu_cloud_key *ck, int form, const uint8_t *ops, const uint32_t *pool_in,
                                 const int32_t *ia, const int32_t *ib, const int32_t *io, uint32_t *pool_out,
                                 int64_t B, void *hip_stream);

/* The same gates without the final key switch (steps 1-4 above): writes
 * the extracted dimension-N samples, which encrypt +-1/8 under the TRLWE
 * key's coefficients. This is the half of a gate that TFHE's MUX runs twice
 * before one key switch (Table "TFHEbenchmark": MUX).
 * out_N: device uint32_t [B][N+1]. Errors as cemu_bootstrap_gates. */
int cemu_blind_rotate_extract(const cemu_cloud_key *ck, int form, const uint8_t *ops, const uint32_t *pool_in,
                              const int32_t *ia, const int32_t *ib, uint32_t *out_N, int64_t B,
                              void *hip_stream);

/* Key switching of B dimension-N samples to dimension n (the last step of
 * a bootstrapped gate; the paper uses it inside the TFHE gate call, Sec. 3).
 * Read as TFHE's key switch: each mask word a'_i is rounded to t * basebit
 * bits (16 in the standard set: add 2^15 and truncate; no rounding when
 * t * basebit = 32), split into t unsigned base-4 digits d_ij,
 * most significant first, and the output is (0, ..., 0, b') minus the rows
 * KS[i][j][d_ij] of the key-switching key, a row with digit 0 subtracting
 * nothing. The phase is preserved up to the key's noise and the rounding.
 * in_N: device [B][N+1]; out_n: device [B][n+1]. Errors: CEMU_ERR_NULL,
 * CEMU_ERR_ALIGN, CEMU_ERR_RANGE (B < 0 or B > 2^40), CEMU_ERR_HIP. */
int cemu_key_switch(const cemu_cloud_key *ck, const uint32_t *in_N, uint32_t *out_n, int64_t B,
                    void *hip_stream);

/* Batched homomorphic multiplexer: out_g = s_g ? a_g : b_g (Table
 * "TFHEbenchmark": MUX, two bootstraps; the FHE MUX select of every stage of
 * the register-mode barrel shifters, Sec. 5.4). Computed as in TFHE: the
 * gates AND(s, a) and ANDNY(s, b) are blind-rotated and extracted without key
 * switching (one batch of 2B blind rotations), their samples are added
 * together with (0, ..., 0, 1/8), and the sum is key-switched once.
 *   pool_in:  device uint32_t [P_in][n+1]
 *   is, ia, ib: device int32_t [B], rows of the selector and of the inputs
 *             chosen when the selector is true (a) or false (b)
 *   io, pool_out, stream, alignment, errors: as cemu_bootstrap_gates.
 * Scratch: the workspaces hold 2B blind-rotation samples. */
int cemu_mux(const cemu_cloud_key *ck, int form, const uint32_t *pool_in, const int32_t *is, const int32_t *ia,
             const int32_t *ib, const int32_t *io, uint32_t *pool_out, int64_t B, void *hip_stream);

/* One circuit level that mixes bootstrapped gates and multiplexers (Table
 * "TFHEbenchmark" gates and MUX; the gates of one level are independent,
 * Sec. 5.2): G gates as cemu_bootstrap_gates and M MUXes as cemu_mux, with
 * all G + 2M blind rotations in one launch and the G + M key switches in
 * another, so a level costs one blind-rotation latency whatever its mix.
 *   pool_in:   device uint32_t [P_in][n+1]
 *   ops, ia, ib: device [G] (uint8_t op codes, int32_t rows), may be NULL
 *             when G = 0
 *   ms, ma, mb: device int32_t [M] rows of the selectors and of the inputs
 *             chosen when the selector is true (ma) or false (mb), may be
 *             NULL when M = 0
 *   io:       device int32_t [G + M] output rows, gates first, then MUXes
 *             (or NULL: output k goes to row k); rows must be distinct
 *   pool_out, stream, alignment: as cemu_bootstrap_gates.
 * Every output equals what cemu_bootstrap_gates (k < G) or cemu_mux
 * (k >= G) computes for the same inputs, bit for bit. G = M = 0 is a no-op.
 * Scratch: the workspaces hold G + 2M blind-rotation samples.
 * Errors: CEMU_ERR_RANGE (G < 0, M < 0, G or M > 2^40, or G + 2M blind
 * rotations beyond one launch, as for cemu_bootstrap_gates), the others as
 * cemu_bootstrap_gates. */
int cemu_bootstrap_level(const cemu_cloud_key *ck, int form, const uint32_t *pool_in, const uint8_t *ops,
                         const int32_t *ia, const int32_t *ib, int64_t G, const int32_t *ms, const int32_t *ma,
                         const int32_t *mb, int64_t M, const int32_t *io, uint32_t *pool_out, void *hip_stream);

/* Unbootstrapped operations of Table "TFHEbenchmark" on a device pool
 * [P][n+1]: NOT (negation of every word), COPY, and CONSTANT (trivial
 * ciphertext (0,...,0, +-1/8)). src, dst: device int32_t [count] rows; for
 * constant, bits is device uint8_t [count]. No key material is needed, only
 * the dimension n (1..CEMU_MAX_LWE_N). Errors: CEMU_ERR_RANGE (count < 0 or
 * count > 2^40), CEMU_ERR_PARAM (n), CEMU_ERR_NULL, CEMU_ERR_HIP. */
int cemu_lwe_not(int32_t n, const uint32_t *pool_in, const int32_t *src, uint32_t *pool_out,
                 const int32_t *dst, int64_t count, void *hip_stream);
int cemu_lwe_copy(int32_t n, const uint32_t *pool_in, const int32_t *src, uint32_t *pool_out,
                  const int32_t *dst, int64_t count, void *hip_stream);
int cemu_lwe_constant(int32_t n, const uint8_t *bits, uint32_t *pool_out, const int32_t *dst, int64_t count,
                      void *hip_stream);

/* Export all key material in the canonical Torus32 layout (host buffers, each
 * may be NULL to skip): lwe_key int32 [n]; tlwe_key int32 [N];
 * bk uint32 [n][2l][2][N] (row c*l+j, component A then B);
 * ksk uint32 [N][t][2^basebit][n+1]. The bootstrapping key is read back from
 * the device (and its int8 limbs recombined), so the export checks the
 * uploaded key. */
int cemu_export_keys(const cemu_secret_key *sk, const cemu_cloud_key *ck, int32_t *lwe_key, int32_t *tlwe_key,
                     uint32_t *bk, uint32_t *ksk);

void cemu_free_secret_key(cemu_secret_key *sk);
void cemu_free_cloud_key(cemu_cloud_key *ck);

/* Launch configuration of the blind-rotation kernels (per cloud key).
 * int8_waves: waves per workgroup of the int8-MFMA kernel, 4 or 8 (default 8).
 * int8_gates_per_wg: gates per workgroup of the int8-MFMA kernel: 16 (default;
 *   the gates fill the MFMA columns and share each streamed key row), or 1: the
 *   latency kernel, one gate per workgroup, for batches too narrow to fill the
 *   GPU (the key limbs fill the columns instead). 0 selects 16.
 * fft_gates_per_wg: gates per workgroup of the FFT64 kernel, 4 (one wave per
 *   SIMD, 512 registers each) or 8 (two waves per SIMD; default), or 1: the
 *   latency kernel, one gate per workgroup of 8 waves (six run the forward
 *   transforms of the six gadget digit rows, two the inverse transforms), for
 *   batches too narrow to fill the GPU.
 * The int8 choices and FFT64 choices 4/8 only change speed, never results.
 * FFT64 choice 1 adds the six digit-row products in another rounding order;
 * since every product is an integer polynomial, all FFT64 choices return the
 * same ciphertexts whenever the transform error stays below half a unit
 * (which is what the parity tests check against the exact oracle).
 * cemu_set_tuning returns CEMU_ERR_PARAM for unsupported values and leaves the
 * key unchanged.
 * Callers: the autotuner (paper_2101_03403_amd/autotune.py). */
typedef struct cemu_tuning {
    int32_t int8_waves;
    int32_t fft_gates_per_wg;
    int32_t int8_gates_per_wg;
    int32_t reserved[5];
} cemu_tuning;
int cemu_get_tuning(const cemu_cloud_key *ck, cemu_tuning *t);
int cemu_set_tuning(cemu_cloud_key *ck, const cemu_tuning *t);

/* Kernel timing with HIP events. While enabled, every kernel the library
 * launches for this cloud key is bracketed by a pair of hipEvents recorded on
 * the same stream. cemu_profile_read waits for the recorded events, returns
 * the summed durations in milliseconds and launch counts per kernel kind, and
 * clears the record. Kinds: 0 = lincomb + modulus switch, 1 = blind rotation
 * (int8), 2 = blind rotation (FFT64), 3 = key switch.
 * ms, launches: host arrays of CEMU_PROFILE_KINDS entries (either may be NULL).
 * Errors: CEMU_ERR_NULL, CEMU_ERR_HIP. */
enum { CEMU_PROFILE_KINDS = 4 };
int cemu_profile_enable(cemu_cloud_key *ck, int enable);
int cemu_profile_read(cemu_cloud_key *ck, double *ms, int64_t *launches);

/* Description of the calling thread's last error ("" if none). */
const char *cemu_last_error(void);

/* Library version string. */
const char *cemu_version(void);

#ifdef __cplusplus
}
#endif
#endif /* CEMU_H */
